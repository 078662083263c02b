// C-ABI runtime of liblz: archive binding and validation, workspace layout,
// error reporting and the entry points that enqueue device work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "lz.h"
#include "lz_internal.h"

static thread_local char g_err[512] = "";

int lz_fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

extern "C" const char* lz_last_error(void) { return g_err; }

// launchers (kernels.hip)
size_t lz_decode_smem_bytes();
int lz_launch_setup(lz_handle* h, hipStream_t s);
int lz_launch_decode_all(lz_handle* h, uint8_t* out, hipStream_t s);
int lz_launch_verify(lz_handle* h, const uint8_t* d_out, uint64_t b0, uint64_t nb, uint64_t* d_tree,
                     void* scratch, hipStream_t s);
int lz_noalloc_setup(int dev, void** ptr);
int lz_decode_occupancy(int* per_cu);
int lz_launch_region_gather(const uint8_t* tmp, uint64_t first, uint64_t offset, uint64_t start,
                            uint64_t nb, uint32_t W, uint32_t LB, uint8_t* out, hipStream_t s);
int lz_launch_requests(lz_handle* h, const lz_request* d_reqs, const uint32_t* d_n, uint64_t n_max,
                       uint64_t single_off, uint64_t single_len, const int64_t* d_ids,
                       uint8_t* d_out, uint64_t cap, uint64_t* d_offsets, void* d_scratch,
                       uint64_t scratch_len, hipStream_t s);

namespace {

inline uint64_t rd64(const uint8_t* p) { uint64_t v; std::memcpy(&v, p, 8); return v; }
inline uint32_t rd32(const uint8_t* p) { uint32_t v; std::memcpy(&v, p, 4); return v; }
inline uint32_t rd16(const uint8_t* p) { uint16_t v; std::memcpy(&v, p, 2); return v; }

uint64_t fnv1a(const uint8_t* p, uint64_t n, uint64_t h) {
  for (uint64_t i = 0; i < n; i++) h = (h ^ p[i]) * kFnvPrime;
  return h;
}

uint32_t width_for(uint64_t n) {
  uint64_t v = n ? n - 1 : 0;
  uint32_t bits = 0;
  while (v) { bits++; v >>= 1; }
  return std::max(1u, (bits + 7) / 8);
}

bool fits(uint64_t off, uint64_t sz, uint64_t len) { return off <= len && sz <= len - off; }

// Header fields and section bounds (magic, version, checksum, ranges,
// n_blocks = ceil(N / B), canonical offset width, section order).
int parse_header(const uint8_t* a, uint64_t len, ArchiveView& v, uint64_t& total) {
  if (len < kHeaderSize) return lz_fail(LZ_EFORMAT, "archive shorter than its header");
  if (std::memcmp(a, "LZAB", 4) || rd16(a + 4) != 2) return lz_fail(LZ_EFORMAT, "bad magic or version");
  if (rd64(a + 120) != fnv1a(a, 120, kFnvBasis)) return lz_fail(LZ_EFORMAT, "header checksum mismatch");
  v = ArchiveView{};
  const uint32_t flags = rd16(a + 6);
  v.block_log2 = a[8];
  const uint32_t D = a[9];
  v.offset_width = a[10];
  v.min_match = a[11];
  v.kind = a[13];
  v.lit_lanes = a[14] + 1u;
  v.seq_lanes = a[15];
  for (int k = 0; k < 4; k++) v.prob_bits[k] = a[16 + k];
  v.n = rd64(a + 24);
  v.n_blocks = rd64(a + 32);
  v.n_reads = rd64(a + 40);
  v.max_record_len = rd32(a + 48);
  v.n_levels = rd32(a + 52);
  v.off_tables = rd64(a + 56);
  v.off_dir = rd64(a + 64);
  v.off_dep_ptr = rd64(a + 72);
  v.off_dep_idx = rd64(a + 80);
  v.off_payload = rd64(a + 88);
  v.off_ridx = rd64(a + 96);
  total = rd64(a + 104);
  if (v.block_log2 < 6 || v.block_log2 > 15 || D < 1 || D > 64) return lz_fail(LZ_EFORMAT, "block size or level cap out of range");
  if (v.seq_lanes < 1 || v.seq_lanes > 64 || v.kind > 2 || v.min_match < 1) return lz_fail(LZ_EFORMAT, "header field out of range");
  for (int k = 0; k < 4; k++)
    if (v.prob_bits[k] < 8 || v.prob_bits[k] > 12) return lz_fail(LZ_EFORMAT, "probability bits out of range");
  if (v.offset_width != width_for(v.n)) return lz_fail(LZ_EFORMAT, "offset width is not canonical");
  if (v.n_blocks != ((v.n + (1ull << v.block_log2) - 1) >> v.block_log2)) return lz_fail(LZ_EFORMAT, "n_blocks != ceil(N/B)");
  if (v.n_blocks >= 0xFFFFFFFFull) return lz_fail(LZ_EFORMAT, "too many blocks");
  if ((flags & 1) != (v.kind == 1 ? 1u : 0u) || (flags & 0xFE)) return lz_fail(LZ_EFORMAT, "flags inconsistent with kind");
  if (v.n_levels > D) return lz_fail(LZ_EFORMAT, "n_levels exceeds the level cap");
  (void)D;
  return LZ_OK;
}

struct Layout {
  uint64_t lut, queue, level_ptr, flags, mark, addr, rqueue, rlevel_ptr, list, ctl, total;
};

Layout layout_for(uint64_t nb) {
  Layout L{};
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) { uint64_t r = o; o = (o + bytes + 255) & ~255ull; return r; };
  L.lut = take(4096 * 4);
  L.queue = take(4 * std::max<uint64_t>(nb, 1));
  L.level_ptr = take(4 * 65);
  L.flags = take(4 * std::max<uint64_t>(nb, 1));
  L.mark = take(4 * std::max<uint64_t>(nb, 1));
  L.addr = take(8 * std::max<uint64_t>(nb, 1));
  L.rqueue = take(4 * std::max<uint64_t>(nb, 1));
  L.rlevel_ptr = take(4 * 130);
  L.list = take(8 * std::max<uint64_t>(nb, 1));
  L.ctl = take(4 * kCtlWords);
  L.total = o;
  return L;
}

int hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) return lz_fail(LZ_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return LZ_OK;
}

}  // namespace

extern "C" int lz_info_get(const uint8_t* a, uint64_t len, lz_info* out) {
  if (!a || !out) return lz_fail(LZ_EINVAL, "lz_info_get: null");
  ArchiveView v;
  uint64_t total = 0;
  int rc = parse_header(a, len, v, total);
  if (rc) return rc;
  std::memset(out, 0, sizeof(*out));
  out->n = v.n;
  out->n_blocks = v.n_blocks;
  out->n_reads = v.n_reads;
  out->archive_len = total;
  out->source_fnv = rd64(a + 112);
  out->workspace_bytes = layout_for(v.n_blocks).total;
  out->block_log2 = v.block_log2;
  out->max_level = a[9];
  out->n_levels = v.n_levels;
  out->offset_width = v.offset_width;
  out->max_record_len = v.max_record_len;
  out->kind = v.kind;
  return LZ_OK;
}

extern "C" int lz_open(const uint8_t* d_archive, uint64_t len, void* d_ws, uint64_t ws_len,
                       hipStream_t s, lz_handle** out) {
  if (!d_archive || !d_ws || !out) return lz_fail(LZ_EINVAL, "lz_open: null argument");
  if (((uintptr_t)d_archive & 15) || ((uintptr_t)d_ws & 255)) return lz_fail(LZ_EINVAL, "lz_open: misaligned archive or workspace");
  *out = nullptr;
  uint8_t hdr[kHeaderSize];
  if (len < kHeaderSize) return lz_fail(LZ_EFORMAT, "archive shorter than its header");
  int rc = hip_check(hipMemcpyAsync(hdr, d_archive, kHeaderSize, hipMemcpyDeviceToHost, s), "lz_open: header copy");
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "lz_open: sync");
  if (rc) return rc;
  ArchiveView v;
  uint64_t total = 0;
  if ((rc = parse_header(hdr, len, v, total))) return rc;
  if (total != len) return lz_fail(LZ_EFORMAT, "archive length %llu != header %llu", (unsigned long long)len, (unsigned long long)total);
  const uint64_t nb = v.n_blocks;
  if (v.off_tables != kHeaderSize || !fits(v.off_tables, kTablesLen, len)) return lz_fail(LZ_EFORMAT, "tables out of bounds");
  if (v.off_dir < v.off_tables + kTablesLen || !fits(v.off_dir, nb * kDirEntry, len)) return lz_fail(LZ_EFORMAT, "directory out of bounds");
  if (v.off_dep_ptr < v.off_dir + nb * kDirEntry || !fits(v.off_dep_ptr, 8 * (nb + 1), len)) return lz_fail(LZ_EFORMAT, "dependency offsets out of bounds");
  // metadata to the host: tables + directory + dependency offsets
  std::vector<uint8_t> meta(v.off_dep_ptr + 8 * (nb + 1));
  rc = hip_check(hipMemcpyAsync(meta.data(), d_archive, meta.size(), hipMemcpyDeviceToHost, s), "lz_open: metadata copy");
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "lz_open: sync");
  if (rc) return rc;
  const uint64_t ndeps = rd64(meta.data() + v.off_dep_ptr + 8 * nb);
  if (v.off_dep_idx < v.off_dep_ptr + 8 * (nb + 1) || !fits(v.off_dep_idx, 4 * ndeps, len)) return lz_fail(LZ_EFORMAT, "dependency list out of bounds");
  if (v.off_payload < v.off_dep_idx + 4 * ndeps || v.off_payload > len || (v.off_payload & 15))
    return lz_fail(LZ_EFORMAT, "payload out of bounds or misaligned");
  std::vector<uint32_t> deps(ndeps);
  if (ndeps) {
    rc = hip_check(hipMemcpyAsync(deps.data(), d_archive + v.off_dep_idx, 4 * ndeps, hipMemcpyDeviceToHost, s), "lz_open: deps copy");
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "lz_open: sync");
    if (rc) return rc;
  }
  const uint64_t pay_end = v.kind == 1 ? v.off_ridx : len;
  if (v.kind == 1) {
    if (v.off_ridx < v.off_payload || !fits(v.off_ridx, 8 * (v.n_reads + 1), len)) return lz_fail(LZ_EFORMAT, "read index out of bounds");
  } else if (v.off_ridx || v.n_reads) {
    return lz_fail(LZ_EFORMAT, "read index present without FASTQ kind");
  }
  // tables sum to 2^P or are empty
  for (int k = 0; k < 4; k++) {
    uint32_t sum = 0;
    for (int q = 0; q < 256; q++) sum += rd16(meta.data() + v.off_tables + 512 * k + 2 * q);
    if (sum != 0 && sum != (1u << v.prob_bits[k])) return lz_fail(LZ_EFORMAT, "frequency table %d does not sum to 2^P", k);
  }
  // directory, dependencies, levels
  const uint32_t D = hdr[9];
  std::vector<uint16_t> lv(nb);
  uint32_t count[kMaxLevels] = {0};
  uint64_t prev_end = 0, lit_total = 0;
  const uint64_t paylen = pay_end - v.off_payload;
  for (uint64_t b = 0; b < nb; b++) {
    const uint8_t* e = meta.data() + v.off_dir + b * kDirEntry;
    const uint64_t po = rd64(e), pl = rd32(e + 8);
    lv[b] = (uint16_t)rd16(e + 20);
    lit_total += rd32(e + 16);
    if (po < prev_end || !fits(po, pl, paylen) || (po & 15)) return lz_fail(LZ_EFORMAT, "block %llu payload out of bounds", (unsigned long long)b);
    prev_end = po + pl;
    if (lv[b] >= D || rd32(e + 12) < 1) return lz_fail(LZ_EFORMAT, "block %llu level or sequence count invalid", (unsigned long long)b);
    const uint64_t d0 = rd64(meta.data() + v.off_dep_ptr + 8 * b), d1 = rd64(meta.data() + v.off_dep_ptr + 8 * (b + 1));
    if ((b == 0 && d0 != 0) || d1 < d0 || d1 > ndeps) return lz_fail(LZ_EFORMAT, "dependency offsets not monotone");
    uint32_t want = 0;
    int64_t last = -1;
    for (uint64_t k = d0; k < d1; k++) {
      const uint32_t d = deps[k];
      if ((int64_t)d <= last || d >= b) return lz_fail(LZ_EFORMAT, "block %llu has an invalid dependency", (unsigned long long)b);
      last = d;
      want = std::max<uint32_t>(want, lv[d] + 1u);
    }
    if (lv[b] != want) return lz_fail(LZ_EFORMAT, "block %llu level %u != %u", (unsigned long long)b, lv[b], want);
    count[lv[b]]++;
  }
  uint32_t n_levels = 0;
  for (uint32_t L = 0; L < kMaxLevels; L++) if (count[L]) n_levels = L + 1;
  if (n_levels != v.n_levels) return lz_fail(LZ_EFORMAT, "n_levels mismatch");
  // device limits of this decoder
  if (v.block_log2 > kMaxBlockLog2) return lz_fail(LZ_EFORMAT, "device decoder supports blocks up to 16 KiB");
  if (v.offset_width > kMaxOffsetWidth) return lz_fail(LZ_EFORMAT, "device decoder supports files below 2^40 bytes");
  if ((1ull << v.block_log2) / v.min_match + 1 > 1025) return lz_fail(LZ_EFORMAT, "device decoder supports at most 1025 sequences per block");
  if (v.kind == 1) {
    std::vector<uint64_t> idx(v.n_reads + 1);
    rc = hip_check(hipMemcpyAsync(idx.data(), d_archive + v.off_ridx, 8 * idx.size(), hipMemcpyDeviceToHost, s), "lz_open: index copy");
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "lz_open: sync");
    if (rc) return rc;
    uint64_t mx = 0;
    if (idx[0] != 0) return lz_fail(LZ_EFORMAT, "read index does not start at 0");
    for (uint64_t r = 0; r < v.n_reads; r++) {
      if (idx[r + 1] <= idx[r]) return lz_fail(LZ_EFORMAT, "read index not increasing");
      mx = std::max(mx, idx[r + 1] - idx[r]);
    }
    if (idx[v.n_reads] != v.n || mx != v.max_record_len) return lz_fail(LZ_EFORMAT, "read index end or max record length wrong");
  }
  const Layout L = layout_for(nb);
  if (ws_len < L.total) return lz_fail(LZ_ECAPACITY, "workspace needs %llu bytes", (unsigned long long)L.total);

  lz_handle* h = new (std::nothrow) lz_handle{};
  if (!h) return lz_fail(LZ_EINVAL, "lz_open: out of host memory");
  v.base = d_archive;
  h->av = v;
  uint8_t* w = (uint8_t*)d_ws;
  h->ws.lut = (uint32_t*)(w + L.lut);
  h->ws.queue = (uint32_t*)(w + L.queue);
  h->ws.level_ptr = (uint32_t*)(w + L.level_ptr);
  h->ws.flags = (uint32_t*)(w + L.flags);
  h->ws.mark = (uint32_t*)(w + L.mark);
  h->ws.addr = (uint64_t*)(w + L.addr);
  h->ws.rqueue = (uint32_t*)(w + L.rqueue);
  h->ws.rlevel_ptr = (uint32_t*)(w + L.rlevel_ptr);
  h->ws.list = (uint64_t*)(w + L.list);
  h->ws.ctl = (uint32_t*)(w + L.ctl);
  std::memcpy(h->level_count, count, sizeof(count));
  h->literal_bytes = lit_total;
  h->payload_bytes = prev_end;
  h->tune.sync_mode = 0;
  h->tune.wg_per_cu = 3;
  h->tune.spin_limit = 0;
  h->tune.req_sync_mode = 0;
  h->tune.plan_blocks = 4096;
  int dev = 0;
  hipDeviceProp_t prop;
  rc = hip_check(hipGetDevice(&dev), "lz_open: device");
  if (!rc) rc = hip_check(hipGetDeviceProperties(&prop, dev), "lz_open: properties");
  if (rc) { delete h; return rc; }
  h->n_cu = prop.multiProcessorCount;
  h->dev = dev;
  {
    int per_cu = 0;
    if ((rc = lz_decode_occupancy(&per_cu))) { delete h; return rc; }
    h->coop_grid = (uint32_t)std::max(1, std::min(per_cu, 3) * h->n_cu);
  }
  {
    void* p = nullptr;   // resolve this device's allocation-free scratch once
    if ((rc = lz_noalloc_setup(dev, &p))) { delete h; return rc; }
  }

  // level-ordered queue of the whole file (ascending block id inside a level)
  std::vector<uint32_t> lptr(65, 0), queue(std::max<uint64_t>(nb, 1));
  for (uint32_t k = 0; k < kMaxLevels; k++) lptr[k + 1] = lptr[k] + count[k];
  {
    std::vector<uint32_t> cur(lptr.begin(), lptr.end() - 1);
    for (uint64_t b = 0; b < nb; b++) queue[cur[lv[b]]++] = (uint32_t)b;
  }
  rc = hip_check(hipMemcpyAsync(h->ws.queue, queue.data(), 4 * queue.size(), hipMemcpyHostToDevice, s), "lz_open: queue upload");
  if (!rc) rc = hip_check(hipMemcpyAsync(h->ws.level_ptr, lptr.data(), 4 * 65, hipMemcpyHostToDevice, s), "lz_open: level upload");
  if (!rc) rc = lz_launch_setup(h, s);
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "lz_open: sync");
  if (rc) { delete h; return rc; }
  *out = h;
  return LZ_OK;
}

extern "C" int lz_close(lz_handle* h) {
  delete h;
  return LZ_OK;
}

extern "C" int lz_get_info(const lz_handle* h, lz_info* out) {
  if (!h || !out) return lz_fail(LZ_EINVAL, "lz_get_info: null");
  std::memset(out, 0, sizeof(*out));
  out->n = h->av.n;
  out->n_blocks = h->av.n_blocks;
  out->n_reads = h->av.n_reads;
  out->workspace_bytes = layout_for(h->av.n_blocks).total;
  out->block_log2 = h->av.block_log2;
  out->n_levels = h->av.n_levels;
  out->offset_width = h->av.offset_width;
  out->max_record_len = h->av.max_record_len;
  out->kind = h->av.kind;
  out->literal_bytes = h->literal_bytes;
  out->payload_bytes = h->payload_bytes;
  return LZ_OK;
}

extern "C" int lz_set_tuning(lz_handle* h, const lz_tuning* t) {
  if (!h || !t) return lz_fail(LZ_EINVAL, "lz_set_tuning: null");
  if (t->sync_mode > 1 || t->wg_per_cu < 1 || t->wg_per_cu > 4 || t->req_sync_mode > 1 || t->plan_blocks > (1u << 20))
    return lz_fail(LZ_EINVAL, "lz_set_tuning: out of range");
  h->tune = *t;
  if (!h->tune.plan_blocks) h->tune.plan_blocks = 4096;
  return LZ_OK;
}

extern "C" int lz_get_tuning(const lz_handle* h, lz_tuning* t) {
  if (!h || !t) return lz_fail(LZ_EINVAL, "lz_get_tuning: null");
  *t = h->tune;
  return LZ_OK;
}

extern "C" int lz_decode_all(lz_handle* h, uint8_t* d_out, uint64_t cap, hipStream_t s) {
  if (!h || (!d_out && h->av.n)) return lz_fail(LZ_EINVAL, "lz_decode_all: null argument");
  if ((uintptr_t)d_out & 15) return lz_fail(LZ_EINVAL, "lz_decode_all: output must be 16-byte aligned");
  if (cap < h->av.n) return lz_fail(LZ_ECAPACITY, "lz_decode_all: output needs %llu bytes", (unsigned long long)h->av.n);
  if (!h->av.n_blocks) return LZ_OK;
  return lz_launch_decode_all(h, d_out, s);
}

extern "C" int lz_sync_status(lz_handle* h, hipStream_t s) {
  if (!h) return lz_fail(LZ_EINVAL, "lz_sync_status: null");
  uint32_t st = 0;
  int rc = hip_check(hipMemcpyAsync(&st, h->ws.ctl + kCtlStatus, 4, hipMemcpyDeviceToHost, s), "lz_sync_status: copy");
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "lz_sync_status: sync");
  if (rc) return rc;
  if (!st) return LZ_OK;
  uint32_t diag[5] = {0, 0, 0, 0, 0};
  rc = hip_check(hipMemcpyAsync(diag, h->ws.ctl + kCtlDiag, sizeof(diag), hipMemcpyDeviceToHost, s), "lz_sync_status: copy");
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "lz_sync_status: sync");
  if (rc) return rc;
  uint32_t zero[6] = {0, 0, 0, 0, 0, 0};
  rc = hip_check(hipMemcpyAsync(h->ws.ctl + kCtlDiag, zero, sizeof(diag), hipMemcpyHostToDevice, s), "lz_sync_status: clear");
  if (!rc) rc = hip_check(hipMemcpyAsync(h->ws.ctl + kCtlStatus, zero, 4, hipMemcpyHostToDevice, s), "lz_sync_status: clear");
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "lz_sync_status: sync");
  if (rc) return rc;
  if (st & kStRange) return lz_fail(LZ_ERANGE, "device: request out of range (status 0x%x)", st);
  if (st & kStCapacity) return lz_fail(LZ_ECAPACITY, "device: scratch or output capacity exhausted (status 0x%x)", st);
  if (st & kStWatchdog)
    return lz_fail(LZ_ECORRUPT, "device: wait timed out (status 0x%x; site %u, %u, %u, seen %u, expected %u)", st,
                   diag[0], diag[1], diag[2], diag[3], diag[4]);
  return lz_fail(LZ_ECORRUPT, "device: decode check failed (status 0x%x)", st);
}

extern "C" int lz_last_stats(lz_handle* h, lz_stats* out, hipStream_t s) {
  if (!h || !out) return lz_fail(LZ_EINVAL, "lz_last_stats: null");
  uint32_t ctl[kCtlPairs + 2];
  int rc = hip_check(hipMemcpyAsync(ctl, h->ws.ctl, sizeof(ctl), hipMemcpyDeviceToHost, s), "lz_last_stats: copy");
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "lz_last_stats: sync");
  if (rc) return rc;
  out->closure_blocks = ctl[kCtlListTail];
  out->scratch_slots = ctl[kCtlSlots];
  out->covering = (uint64_t)ctl[kCtlPairs] | ((uint64_t)ctl[kCtlPairs + 1] << 32);
  return LZ_OK;
}

extern "C" int lz_verify(lz_handle* h, const uint8_t* d_out, uint64_t* d_tree, void* d_scratch,
                         uint64_t scratch_len, hipStream_t s) {
  if (!h || !d_tree || (!d_out && h->av.n)) return lz_fail(LZ_EINVAL, "lz_verify: null argument");
  if (scratch_len < 8 * h->av.n_blocks || (!d_scratch && h->av.n_blocks)) return lz_fail(LZ_ECAPACITY, "lz_verify: scratch needs %llu bytes", (unsigned long long)(8 * h->av.n_blocks));
  return lz_launch_verify(h, d_out, 0, h->av.n_blocks, d_tree, d_scratch, s);
}

extern "C" int lz_verify_range(lz_handle* h, const uint8_t* d_out, uint64_t offset, uint64_t len,
                               void* d_scratch, uint64_t scratch_len, hipStream_t s) {
  if (!h) return lz_fail(LZ_EINVAL, "lz_verify_range: null handle");
  const uint64_t N = h->av.n, B = 1ull << h->av.block_log2;
  if (offset > N || len > N - offset) return lz_fail(LZ_ERANGE, "lz_verify_range: range outside the file");
  if (!len) return LZ_OK;
  if (!d_out) return lz_fail(LZ_EINVAL, "lz_verify_range: null output");
  if (offset % B || (offset + len != N && len % B))
    return lz_fail(LZ_EINVAL, "lz_verify_range: range must cover whole blocks");
  const uint64_t nb = (len + B - 1) / B;
  if (scratch_len < 8 * nb || !d_scratch) return lz_fail(LZ_ECAPACITY, "lz_verify_range: scratch needs %llu bytes", (unsigned long long)(8 * nb));
  return lz_launch_verify(h, d_out, offset / B, nb, nullptr, d_scratch, s);
}

extern "C" int lz_decode_range(lz_handle* h, uint64_t offset, uint64_t len, uint8_t* d_out,
                               void* d_scratch, uint64_t scratch_len, hipStream_t s) {
  if (!h) return lz_fail(LZ_EINVAL, "lz_decode_range: null handle");
  if (offset > h->av.n || len > h->av.n - offset) return lz_fail(LZ_ERANGE, "lz_decode_range: [%llu, +%llu) outside N = %llu", (unsigned long long)offset, (unsigned long long)len, (unsigned long long)h->av.n);
  if (!len) return LZ_OK;
  if (!d_out) return lz_fail(LZ_EINVAL, "lz_decode_range: null output");
  return lz_launch_requests(h, nullptr, nullptr, 1, offset, len, nullptr, d_out, len, nullptr, d_scratch, scratch_len, s);
}

extern "C" int lz_read_lookup(lz_handle* h, const int64_t* d_ids, uint64_t n, uint8_t* d_out,
                              uint64_t cap, uint64_t* d_offsets, void* d_scratch,
                              uint64_t scratch_len, hipStream_t s) {
  if (!h) return lz_fail(LZ_EINVAL, "lz_read_lookup: null handle");
  if (h->av.kind != 1) return lz_fail(LZ_ENOINDEX, "lz_read_lookup: archive has no read index");
  if (!n) return LZ_OK;
  if (!d_ids || !d_out || !d_offsets) return lz_fail(LZ_EINVAL, "lz_read_lookup: null argument");
  if (cap < n * (uint64_t)h->av.max_record_len) return lz_fail(LZ_ECAPACITY, "lz_read_lookup: output needs %llu bytes", (unsigned long long)(n * (uint64_t)h->av.max_record_len));
  return lz_launch_requests(h, nullptr, nullptr, n, 0, 0, d_ids, d_out, cap, d_offsets, d_scratch, scratch_len, s);
}

extern "C" int lz_decode_batch(lz_handle* h, const lz_request* d_reqs, const uint32_t* d_n, uint64_t n_max,
                               uint8_t* d_out, uint64_t cap, uint64_t* d_offsets, void* d_scratch,
                               uint64_t scratch_len, hipStream_t s) {
  if (!h || !d_reqs || !d_n || !d_out || !d_offsets) return lz_fail(LZ_EINVAL, "lz_decode_batch: null argument");
  if (!n_max) return LZ_OK;
  return lz_launch_requests(h, d_reqs, d_n, n_max, 0, 0, nullptr, d_out, cap, d_offsets, d_scratch, scratch_len, s);
}

extern "C" int lz_decode_region(lz_handle* h, const lz_fasta_seq* sq, uint64_t start, uint64_t end,
                                uint8_t* d_out, void* d_scratch, uint64_t scratch_len, hipStream_t s) {
  if (!h || !sq) return lz_fail(LZ_EINVAL, "lz_decode_region: null argument");
  if (start > end || end > sq->length) return lz_fail(LZ_ERANGE, "lz_decode_region: [%llu, %llu) outside the sequence of %llu bases", (unsigned long long)start, (unsigned long long)end, (unsigned long long)sq->length);
  if (!sq->line_bases || sq->line_bytes != sq->line_bases + 1u)
    return lz_fail(LZ_ENOINDEX, "lz_decode_region: sequence has uneven lines");
  if (start == end) return LZ_OK;
  if (!d_out || !d_scratch) return lz_fail(LZ_EINVAL, "lz_decode_region: null buffer");
  const uint64_t W = sq->line_bases, LB = sq->line_bytes;
  auto pos = [&](uint64_t k) { return sq->offset + (k / W) * LB + k % W; };
  const uint64_t first = pos(start), last = pos(end - 1) + 1;
  if (last > h->av.n) return lz_fail(LZ_ERANGE, "lz_decode_region: sequence lies outside the file");
  const uint64_t span = last - first, head = (span + 255) & ~255ull;
  if (((uintptr_t)d_scratch & 255) || scratch_len < head) return lz_fail(LZ_ECAPACITY, "lz_decode_region: scratch needs more than %llu bytes", (unsigned long long)head);
  uint8_t* tmp = reinterpret_cast<uint8_t*>(d_scratch);
  int rc = lz_decode_range(h, first, span, tmp, tmp + head, scratch_len - head, s);
  if (rc) return rc;
  return lz_launch_region_gather(tmp, first, sq->offset, start, end - start, (uint32_t)W, (uint32_t)LB, d_out, s);
}
