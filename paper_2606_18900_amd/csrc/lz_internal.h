// Internal definitions shared by the library's host and device sources:
// container format v2 layout constants, the handle, and error reporting.
#pragma once
#include <cstdint>

#include "lz.h"

constexpr uint64_t kHeaderSize = 128;
constexpr uint64_t kTablesLen = 4 * 256 * 2;   // 4 tables of 256 u16 frequencies
constexpr uint64_t kDirEntry = 32;             // payload_off u64, payload_len u32,
                                               // n_seq u32, n_lit u32, level u16,
                                               // reserved u16, block_fnv u64
constexpr uint64_t kFnvBasis = 0xcbf29ce484222325ull;
constexpr uint64_t kFnvPrime = 0x00000100000001b3ull;

enum StreamKind { kLit = 0, kCmd = 1, kMlen = 2, kOff = 3 };
enum StreamMode { kModeEmpty = 0, kModeConst = 1, kModeRaw = 2, kModeRans = 3 };

// device limits of the decoder
constexpr uint32_t kMaxBlockLog2 = 14;
constexpr uint32_t kMaxPLit = 12;
constexpr uint32_t kMaxPSeq = 12;
constexpr uint32_t kMaxOffsetWidth = 5;   // absolute offsets below 2^40
constexpr uint32_t kMaxLevels = 64;

// status bits latched by kernels in the workspace status word
enum : uint32_t {
  kStCorrupt = 1u,     // payload failed a decode check
  kStCapacity = 2u,    // scratch slots or output capacity exhausted
  kStRange = 4u,       // request outside the file / read id out of range
  kStWatchdog = 8u,    // a dependency wait exceeded the spin limit
  kStHash = 16u,       // FNV verification mismatch
};

int lz_fail(int code, const char* fmt, ...);

// Everything a kernel needs to find an archive's sections in device memory.
struct ArchiveView {
  const uint8_t* base;     // device
  uint64_t n, n_blocks, n_reads;
  uint64_t off_tables, off_dir, off_dep_ptr, off_dep_idx, off_payload, off_ridx;
  uint32_t block_log2, offset_width, min_match, lit_lanes, seq_lanes;
  uint32_t prob_bits[4];
  uint32_t n_levels, max_record_len, kind;
};

// Workspace carve-up (device pointers), see lz_open.
struct Workspace {
  uint32_t* lut;          // 4096 packed literal decode entries
  uint32_t* queue;        // n_blocks: whole-file level-ordered block ids
  uint32_t* level_ptr;    // 65: level offsets into queue
  uint32_t* flags;        // n_blocks: completion epoch per block
  uint32_t* mark;         // n_blocks: request epoch per block (closure)
  uint64_t* addr;         // n_blocks: device address of decoded block bytes
  uint32_t* rqueue;       // n_blocks: request closure queue (level order)
  uint32_t* rlevel_ptr;   // 65 level offsets + 64 cursors of rqueue
  uint64_t* list;         // n_blocks: closure work list, entries (epoch << 32 | block)
  uint32_t* ctl;          // control words (see kCtl*)
};

// control words in Workspace::ctl (u32 each; 64-bit values use two words)
enum : uint32_t {
  kCtlStatus = 0,     // latched status bits
  kCtlTicket = 1,     // cooperative decode: grid-barrier arrivals
  kCtlEpoch = 2,      // completion epoch (per-block flags)
  kCtlREpoch = 3,     // request epoch (closure marks)
  kCtlListTail = 4,   // closure list: entries pushed
  kCtlListHead = 5,   // closure list: entries taken
  kCtlListDone = 6,   // closure list: entries fully expanded
  kCtlSlots = 7,      // scratch slots handed out
  kCtlNReq = 8,       // number of requests of the current batch
  kCtlTotal = 10,     // u64: total output bytes of the batch
  kCtlPairs = 12,     // u64: (request, covering block) pairs of the batch
  kCtlLevelCnt = 16,  // 64 level counters of the closure queue
  kCtlDiag = 80,      // first watchdog: site, block, dependency, seen, expected
  kCtlClock = 96,     // u64[16]: stage clocks of an instrumented build (LZ_STAGE_CLOCKS)
  kCtlWords = 128,
};

struct lz_handle {
  ArchiveView av;
  Workspace ws;
  lz_tuning tune;
  int n_cu;
  int dev;                            // device the handle was opened on
  uint32_t coop_grid;                 // resident decode workgroups (cooperative launch)
  uint32_t level_count[kMaxLevels];   // host copy of the whole-file level histogram
  uint64_t literal_bytes;             // sum of n_lit over blocks
  uint64_t payload_bytes;             // end of the last block payload
};
