// Stream-separated FASTQ container (paper, Discussion: "Where ACEAPEX Stands
// on Ratio" -- read ids, sequences and quality strings stored apart, each
// group homogeneous, the codec unchanged).
//
// A 4-line FASTQ file becomes four line streams, each one ordinary archive of
// this codec (kind 0): H (id lines), S (sequence lines), P ('+' lines), Q
// (quality lines), every line with its newline.  Records are reassembled
// through a read index: hstart[i], sstart[i] are the offsets of record i's id
// and sequence lines in H and S.  Only files whose third lines are a bare '+'
// and whose quality lines are as long as their sequence lines are taken, so
// record i's P and Q lines start at 2 i and sstart[i], and its first byte in
// the file is hstart[i] + 2 sstart[i] + 2 i.
//
// Container (little-endian):
//    0 "LZSF"   4 u16 version 2   6 u16 flags 3   8 u64 N   16 u64 n_reads
//   24 u64 offset of hstart[]   32 u64 offset of sstart[]   (n_reads+1 u64 each)
//   40 u64 stream archive offsets[4] (multiples of 256)   72 u64 lengths[4]
//  104 u64 FNV-1a-64 of the source   112 u32 longest record   116 u32 0
//  120 u64 FNV-1a-64 of bytes 0..119
//  128 hstart[], sstart[], then the four archives; gaps are zero bytes.
//
// Device side: each stream is decoded by its own lz_handle (whole file,
// range or batched requests); the kernels here put the lines back in record
// order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "lz.h"
#include "lz_internal.h"

namespace {

constexpr uint64_t kSplitHeader = 128;
constexpr uint32_t kSplitVersion = 2, kSplitFlags = 3;
constexpr uint32_t kJoinWG = 256;               // one wave per record

uint64_t rd64(const uint8_t* p) { uint64_t v; std::memcpy(&v, p, 8); return v; }
uint32_t rd32(const uint8_t* p) { uint32_t v; std::memcpy(&v, p, 4); return v; }
void wr64(uint8_t* p, uint64_t v) { std::memcpy(p, &v, 8); }
uint64_t pad256(uint64_t v) { return (v + 255) & ~255ull; }

uint64_t fnv(const uint8_t* p, uint64_t n, uint64_t h = kFnvBasis) {
  for (uint64_t i = 0; i < n; i++) h = (h ^ p[i]) * kFnvPrime;
  return h;
}

int hip_ok(hipError_t e, const char* what) {
  return e == hipSuccess ? LZ_OK : lz_fail(LZ_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

struct Head {
  uint64_t n, n_reads, off_h, off_s, sub_off[4], sub_len[4], src_fnv;
  uint32_t max_rec;
};

int parse_head(const uint8_t* a, uint64_t len, Head& h) {
  if (len < kSplitHeader || std::memcmp(a, "LZSF", 4)) return lz_fail(LZ_EFORMAT, "not a split FASTQ container");
  uint16_t ver, fl;
  std::memcpy(&ver, a + 4, 2);
  std::memcpy(&fl, a + 6, 2);
  if (ver != kSplitVersion || fl != kSplitFlags) return lz_fail(LZ_EFORMAT, "split container: unsupported version or flags");
  if (rd64(a + 120) != fnv(a, 120)) return lz_fail(LZ_EFORMAT, "split container: header hash mismatch");
  h.n = rd64(a + 8);
  h.n_reads = rd64(a + 16);
  h.off_h = rd64(a + 24);
  h.off_s = rd64(a + 32);
  for (int k = 0; k < 4; k++) {
    h.sub_off[k] = rd64(a + 40 + 8 * k);
    h.sub_len[k] = rd64(a + 72 + 8 * k);
  }
  h.src_fnv = rd64(a + 104);
  h.max_rec = rd32(a + 112);
  const uint64_t tab = 8 * (h.n_reads + 1);
  if (h.n_reads > (len >> 4) || h.off_h < kSplitHeader || h.off_s < h.off_h + tab || h.off_s + tab > len)
    return lz_fail(LZ_EFORMAT, "split container: record tables out of bounds");
  uint64_t prev = h.off_s + tab;
  for (int k = 0; k < 4; k++) {
    if ((h.sub_off[k] & 255) || h.sub_off[k] < prev || h.sub_len[k] > len - h.sub_off[k])
      return lz_fail(LZ_EFORMAT, "split container: stream archive %d out of bounds", k);
    prev = h.sub_off[k] + h.sub_len[k];
  }
  return LZ_OK;
}

// ---- kernels ---------------------------------------------------------------

struct JoinArgs {
  const uint64_t* hs;      // hstart[] (device)
  const uint64_t* ss;      // sstart[] (device)
  const uint8_t* src[4];   // where stream k's byte at offset base[k] lies
  uint64_t base[4];
  uint64_t r0, r1;         // records [r0, r1)
  uint64_t lo, hi;         // file bytes [lo, hi) go to out[0 .. hi - lo)
  uint8_t* out;
};

// Records [r0, r1) back in file order, clipped to [lo, hi): one wave per
// record (grid-stride), each line copied byte by byte with consecutive lanes
// on consecutive bytes.
__global__ void __launch_bounds__(kJoinWG) k_split_join(JoinArgs J) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t waves = (uint64_t)gridDim.x * (kJoinWG / 64);
  for (uint64_t i = J.r0 + (uint64_t)blockIdx.x * (kJoinWG / 64) + (threadIdx.x >> 6); i < J.r1; i += waves) {
    const uint64_t h0 = J.hs[i], h1 = J.hs[i + 1], s0 = J.ss[i], s1 = J.ss[i + 1];
    uint64_t pos = h0 + 2 * s0 + 2 * i;                 // the record's first byte in the file
    const uint64_t beg[4] = {h0, s0, 2 * i, s0};
    const uint64_t len[4] = {h1 - h0, s1 - s0, 2, s1 - s0};
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const uint8_t* src = J.src[k] + (beg[k] - J.base[k]);
      const uint64_t a = max(pos, J.lo), b = min(pos + len[k], J.hi);
      for (uint64_t p = a + lane; p < b; p += 64) J.out[p - J.lo] = src[p - pos];
      pos += len[k];
    }
  }
}

struct ReqPlan {
  const uint64_t* hs;
  const uint64_t* ss;
  const int64_t* ids;
  uint64_t n, n_reads;
  lz_request* reqs[4];     // one range request per id and stream
  uint32_t* d_n;
};

// Per id, the byte range of each of its four lines in its stream.  An id
// outside [0, n_reads) becomes an invalid range, which the stream's request
// kernels latch as LZ_ERANGE.
__global__ void k_split_reqs(ReqPlan P) {
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0) *P.d_n = (uint32_t)P.n;
  if (k >= P.n) return;
  const int64_t r = P.ids[k];
  if (r < 0 || (uint64_t)r >= P.n_reads) {
    for (int j = 0; j < 4; j++) P.reqs[j][k] = lz_request{1, -1, 0};
    return;
  }
  const uint64_t i = (uint64_t)r;
  const uint64_t h0 = P.hs[i], h1 = P.hs[i + 1], s0 = P.ss[i], s1 = P.ss[i + 1];
  P.reqs[0][k] = lz_request{1, (int64_t)h0, (int64_t)(h1 - h0)};
  P.reqs[1][k] = lz_request{1, (int64_t)s0, (int64_t)(s1 - s0)};
  P.reqs[2][k] = lz_request{1, (int64_t)(2 * i), 2};
  P.reqs[3][k] = lz_request{1, (int64_t)s0, (int64_t)(s1 - s0)};
}

struct GatherArgs {
  const uint8_t* piece[4];      // each stream's batch output
  const uint64_t* poff[4];      // its n + 1 offsets
  uint64_t n;
  uint8_t* out;
  uint64_t* offsets;            // n + 1: record k at out[offsets[k] .. offsets[k+1])
};

// Record k = its four lines from the streams' batch outputs; one wave per
// record (grid-stride).
__global__ void __launch_bounds__(kJoinWG) k_split_gather(GatherArgs G) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t waves = (uint64_t)gridDim.x * (kJoinWG / 64);
  for (uint64_t k = (uint64_t)blockIdx.x * (kJoinWG / 64) + (threadIdx.x >> 6); k <= G.n; k += waves) {
    uint64_t o = G.poff[0][k] + G.poff[1][k] + G.poff[2][k] + G.poff[3][k];
    if (lane == 0) G.offsets[k] = o;
    if (k == G.n) continue;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const uint64_t a = G.poff[j][k], len = G.poff[j][k + 1] - a;
      for (uint64_t p = lane; p < len; p += 64) G.out[o + p] = G.piece[j][a + p];
      o += len;
    }
  }
}

}  // namespace

// ---- handle ------------------------------------------------------------------

struct lz_split {
  Head hd;
  lz_handle* sub[4] = {nullptr, nullptr, nullptr, nullptr};
  uint8_t* buf = nullptr;             // workspace: the four decoded streams
  uint64_t base[4] = {0, 0, 0, 0};    // stream k at buf + base[k]
  uint64_t slen[4] = {0, 0, 0, 0};    // decoded stream lengths
  uint64_t maxpiece[4] = {0, 0, 0, 0};
  uint64_t nblocks[4] = {0, 0, 0, 0};
  uint32_t block_log2[4] = {0, 0, 0, 0};
  const uint64_t* d_hs = nullptr;
  const uint64_t* d_ss = nullptr;
  std::vector<uint64_t> hs, ss;       // host copies of the record tables
  uint32_t grid = 1;
};

namespace {

// Workspace: the stream buffer, then each stream handle's workspace.
struct SplitLayout {
  uint64_t base[4], ws[4], total;
};

SplitLayout split_layout(const uint64_t slen[4], const uint64_t wsb[4]) {
  SplitLayout L;
  uint64_t o = 0;
  for (int k = 0; k < 4; k++) { L.base[k] = o; o = pad256(o + slen[k]); }
  for (int k = 0; k < 4; k++) { L.ws[k] = o; o = pad256(o + std::max<uint64_t>(wsb[k], 256)); }
  L.total = o;
  return L;
}

// Headers of the container and of its four stream archives, from device memory.
int read_heads(const uint8_t* d, uint64_t len, hipStream_t s, Head& h, lz_info sub[4]) {
  uint8_t a[kSplitHeader];
  if (len < kSplitHeader) return lz_fail(LZ_EFORMAT, "split container shorter than its header");
  int rc = hip_ok(hipMemcpyAsync(a, d, kSplitHeader, hipMemcpyDeviceToHost, s), "split: header copy");
  if (!rc) rc = hip_ok(hipStreamSynchronize(s), "split: sync");
  if (!rc) rc = parse_head(a, len, h);
  for (int k = 0; !rc && k < 4; k++) {
    uint8_t b[kHeaderSize];
    if (h.sub_len[k] < kHeaderSize) return lz_fail(LZ_EFORMAT, "split container: stream archive %d too short", k);
    rc = hip_ok(hipMemcpyAsync(b, d + h.sub_off[k], kHeaderSize, hipMemcpyDeviceToHost, s), "split: stream header copy");
    if (!rc) rc = hip_ok(hipStreamSynchronize(s), "split: sync");
    if (!rc) rc = lz_info_get(b, h.sub_len[k], &sub[k]);
    if (!rc && sub[k].kind != 0) rc = lz_fail(LZ_EFORMAT, "split container: stream archive %d is not kind 0", k);
  }
  return rc;
}

// Scratch of one stream's request call for n requests (spans, prefix sums,
// then one slot per block: a bound on any closure).
uint64_t req_scratch(const lz_split* sp, int k, uint64_t n) {
  n = std::max<uint64_t>(n, 1);
  return ((16 * n + 16 * (n + 1) + 255) & ~255ull) + sp->nblocks[k] * (1ull << sp->block_log2[k]);
}

}  // namespace

extern "C" int lz_encode_split(const uint8_t* x, uint64_t n, const lz_params* p, uint8_t** out,
                               uint64_t* out_len) {
  if (!p || !out || !out_len || (n && !x)) return lz_fail(LZ_EINVAL, "lz_encode_split: null argument");
  *out = nullptr;
  *out_len = 0;
  if (n && x[n - 1] != '\n') return lz_fail(LZ_EINVAL, "lz_encode_split: FASTQ text must end with a newline");
  // lines, four per record
  std::vector<uint64_t> ls;                 // line starts, then n
  for (uint64_t i = 0; i < n;) {
    ls.push_back(i);
    const void* q = std::memchr(x + i, '\n', n - i);
    i = (uint64_t)((const uint8_t*)q - x) + 1;
  }
  if (ls.size() % 4) return lz_fail(LZ_EINVAL, "lz_encode_split: FASTQ text must hold whole 4-line records");
  ls.push_back(n);
  const uint64_t nr = (ls.size() - 1) / 4;
  std::vector<uint8_t> st[4];
  std::vector<uint64_t> hs(nr + 1, 0), ss(nr + 1, 0);
  uint32_t longest = 0;
  for (uint64_t r = 0; r < nr; r++) {
    const uint64_t* l = &ls[4 * r];
    const uint64_t len[4] = {l[1] - l[0], l[2] - l[1], l[3] - l[2], l[4] - l[3]};   // with newlines
    if (x[l[0]] != '@') return lz_fail(LZ_EINVAL, "lz_encode_split: record %llu: id line lacks '@'", (unsigned long long)r);
    if (len[2] != 2 || x[l[2]] != '+') return lz_fail(LZ_EINVAL, "lz_encode_split: record %llu: third line is not a bare '+'", (unsigned long long)r);
    if (len[3] != len[1]) return lz_fail(LZ_EINVAL, "lz_encode_split: record %llu: quality and sequence lengths differ", (unsigned long long)r);
    for (int k = 0; k < 4; k++) st[k].insert(st[k].end(), x + l[k], x + l[k] + len[k]);
    hs[r + 1] = hs[r] + len[0];
    ss[r + 1] = ss[r] + len[1];
    longest = (uint32_t)std::max<uint64_t>(longest, l[4] - l[0]);
  }
  lz_params q = *p;
  q.kind = 0;
  uint8_t* sub[4] = {nullptr, nullptr, nullptr, nullptr};
  uint64_t sublen[4] = {0, 0, 0, 0};
  int rc = LZ_OK;
  for (int k = 0; k < 4 && !rc; k++) rc = lz_encode(st[k].data(), st[k].size(), &q, &sub[k], &sublen[k]);
  if (rc) {
    for (auto* a : sub) lz_free(a);
    return rc;
  }
  const uint64_t off_h = kSplitHeader, off_s = off_h + 8 * (nr + 1);
  uint64_t sub_off[4], o = pad256(off_s + 8 * (nr + 1));
  for (int k = 0; k < 4; k++) { sub_off[k] = o; o = pad256(o + sublen[k]); }
  const uint64_t total = sub_off[3] + sublen[3];
  uint8_t* buf = (uint8_t*)std::calloc(total, 1);
  if (!buf) {
    for (auto* a : sub) lz_free(a);
    return lz_fail(LZ_EINVAL, "lz_encode_split: out of host memory");
  }
  std::memcpy(buf, "LZSF", 4);
  const uint16_t ver = kSplitVersion, fl = kSplitFlags;
  std::memcpy(buf + 4, &ver, 2);
  std::memcpy(buf + 6, &fl, 2);
  wr64(buf + 8, n);
  wr64(buf + 16, nr);
  wr64(buf + 24, off_h);
  wr64(buf + 32, off_s);
  for (int k = 0; k < 4; k++) { wr64(buf + 40 + 8 * k, sub_off[k]); wr64(buf + 72 + 8 * k, sublen[k]); }
  wr64(buf + 104, fnv(x, n));
  std::memcpy(buf + 112, &longest, 4);
  wr64(buf + 120, fnv(buf, 120));
  std::memcpy(buf + off_h, hs.data(), 8 * (nr + 1));
  std::memcpy(buf + off_s, ss.data(), 8 * (nr + 1));
  for (int k = 0; k < 4; k++) {
    std::memcpy(buf + sub_off[k], sub[k], sublen[k]);
    lz_free(sub[k]);
  }
  *out = buf;
  *out_len = total;
  return LZ_OK;
}

extern "C" int lz_split_info_get(const uint8_t* d_container, uint64_t len, hipStream_t s, lz_split_info* out) {
  if (!d_container || !out) return lz_fail(LZ_EINVAL, "lz_split_info_get: null argument");
  Head h;
  lz_info sub[4];
  int rc = read_heads(d_container, len, s, h, sub);
  if (rc) return rc;
  std::memset(out, 0, sizeof(*out));
  uint64_t slen[4], wsb[4];
  for (int k = 0; k < 4; k++) {
    slen[k] = out->stream_len[k] = sub[k].n;
    out->archive_len[k] = h.sub_len[k];
    wsb[k] = sub[k].workspace_bytes;
  }
  out->n = h.n;
  out->n_reads = h.n_reads;
  out->container_len = h.sub_off[3] + h.sub_len[3];
  out->source_fnv = h.src_fnv;
  out->workspace_bytes = split_layout(slen, wsb).total;
  out->max_record_len = h.max_rec;
  return LZ_OK;
}

extern "C" int lz_split_open(const uint8_t* d_container, uint64_t len, void* d_ws, uint64_t ws_len,
                             hipStream_t s, lz_split** out) {
  if (!d_container || !d_ws || !out) return lz_fail(LZ_EINVAL, "lz_split_open: null argument");
  if (((uintptr_t)d_container & 255) || ((uintptr_t)d_ws & 255)) return lz_fail(LZ_EINVAL, "lz_split_open: misaligned container or workspace");
  *out = nullptr;
  Head h;
  lz_info sub[4];
  int rc = read_heads(d_container, len, s, h, sub);
  if (rc) return rc;
  if (h.sub_off[3] + h.sub_len[3] != len) return lz_fail(LZ_EFORMAT, "split container length %llu != %llu", (unsigned long long)len, (unsigned long long)(h.sub_off[3] + h.sub_len[3]));
  uint64_t slen[4], wsb[4];
  for (int k = 0; k < 4; k++) { slen[k] = sub[k].n; wsb[k] = sub[k].workspace_bytes; }
  const SplitLayout L = split_layout(slen, wsb);
  if (ws_len < L.total) return lz_fail(LZ_ECAPACITY, "lz_split_open: workspace needs %llu bytes", (unsigned long long)L.total);
  lz_split* sp = new (std::nothrow) lz_split{};
  if (!sp) return lz_fail(LZ_EINVAL, "lz_split_open: out of host memory");
  sp->hd = h;
  // record tables: to the host, checked against the stream lengths and N
  const uint64_t nr = h.n_reads;
  sp->hs.resize(nr + 1);
  sp->ss.resize(nr + 1);
  rc = hip_ok(hipMemcpyAsync(sp->hs.data(), d_container + h.off_h, 8 * (nr + 1), hipMemcpyDeviceToHost, s), "split: table copy");
  if (!rc) rc = hip_ok(hipMemcpyAsync(sp->ss.data(), d_container + h.off_s, 8 * (nr + 1), hipMemcpyDeviceToHost, s), "split: table copy");
  if (!rc) rc = hip_ok(hipStreamSynchronize(s), "split: sync");
  if (rc) { delete sp; return rc; }
  uint64_t longest = 0;
  if (sp->hs[0] || sp->ss[0]) rc = lz_fail(LZ_EFORMAT, "split container: record tables do not start at 0");
  for (uint64_t i = 0; i < nr && !rc; i++) {
    const uint64_t hl = sp->hs[i + 1] - sp->hs[i], sl = sp->ss[i + 1] - sp->ss[i];
    if (sp->hs[i + 1] <= sp->hs[i] || sp->ss[i + 1] <= sp->ss[i]) rc = lz_fail(LZ_EFORMAT, "split container: record tables not increasing");
    sp->maxpiece[0] = std::max(sp->maxpiece[0], hl);
    sp->maxpiece[1] = std::max(sp->maxpiece[1], sl);
    longest = std::max(longest, hl + 2 * sl + 2);
  }
  sp->maxpiece[2] = 2;
  sp->maxpiece[3] = sp->maxpiece[1];
  if (!rc && (sp->hs[nr] != slen[0] || sp->ss[nr] != slen[1] || 2 * nr != slen[2] || sp->ss[nr] != slen[3] ||
              sp->hs[nr] + 2 * sp->ss[nr] + 2 * nr != h.n || longest != h.max_rec))
    rc = lz_fail(LZ_EFORMAT, "split container: record tables disagree with the streams");
  if (rc) { delete sp; return rc; }
  uint8_t* w = (uint8_t*)d_ws;
  sp->buf = w;
  for (int k = 0; k < 4 && !rc; k++) {
    sp->base[k] = L.base[k];
    sp->slen[k] = slen[k];
    sp->nblocks[k] = sub[k].n_blocks;
    sp->block_log2[k] = sub[k].block_log2;
    rc = lz_open(d_container + h.sub_off[k], h.sub_len[k], w + L.ws[k], std::max<uint64_t>(wsb[k], 256), s, &sp->sub[k]);
  }
  if (rc) { lz_split_close(sp); return rc; }
  sp->d_hs = reinterpret_cast<const uint64_t*>(d_container + h.off_h);
  sp->d_ss = reinterpret_cast<const uint64_t*>(d_container + h.off_s);
  int dev = 0, ncu = 0;
  rc = hip_ok(hipGetDevice(&dev), "split: device");
  if (!rc) rc = hip_ok(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev), "split: CUs");
  if (rc) { lz_split_close(sp); return rc; }
  sp->grid = (uint32_t)std::max(1, 8 * ncu);
  *out = sp;
  return LZ_OK;
}

extern "C" int lz_split_close(lz_split* sp) {
  if (!sp) return LZ_OK;
  for (auto* h : sp->sub) if (h) lz_close(h);
  delete sp;
  return LZ_OK;
}

extern "C" int lz_split_stream(lz_split* sp, uint32_t k, lz_handle** out) {
  if (!sp || !out || k > 3) return lz_fail(LZ_EINVAL, "lz_split_stream: bad argument");
  *out = sp->sub[k];
  return LZ_OK;
}

namespace {

// Records [r0, r1) clipped to file bytes [lo, hi) into out, stream k's byte at
// offset beg[k] lying at buf + base[k].
int launch_join(lz_split* sp, uint64_t r0, uint64_t r1, const uint64_t beg[4], uint64_t lo, uint64_t hi,
                uint8_t* out, hipStream_t s) {
  if (r1 <= r0 || hi <= lo) return LZ_OK;
  JoinArgs J{};
  J.hs = sp->d_hs;
  J.ss = sp->d_ss;
  for (int k = 0; k < 4; k++) { J.src[k] = sp->buf + sp->base[k]; J.base[k] = beg[k]; }
  J.r0 = r0;
  J.r1 = r1;
  J.lo = lo;
  J.hi = hi;
  J.out = out;
  const uint64_t need = (r1 - r0 + kJoinWG / 64 - 1) / (kJoinWG / 64);
  const uint32_t grid = (uint32_t)std::min<uint64_t>(need, sp->grid);
  hipLaunchKernelGGL(k_split_join, dim3(grid), dim3(kJoinWG), 0, s, J);
  return hip_ok(hipGetLastError(), "k_split_join");
}

}  // namespace

extern "C" int lz_split_decode_all(lz_split* sp, uint8_t* d_out, uint64_t cap, hipStream_t s) {
  if (!sp || (!d_out && sp->hd.n)) return lz_fail(LZ_EINVAL, "lz_split_decode_all: null argument");
  if (cap < sp->hd.n) return lz_fail(LZ_ECAPACITY, "lz_split_decode_all: output needs %llu bytes", (unsigned long long)sp->hd.n);
  for (int k = 0; k < 4; k++) {
    if (!sp->slen[k]) continue;
    const int rc = lz_decode_all(sp->sub[k], sp->buf + sp->base[k], sp->slen[k], s);
    if (rc) return rc;
  }
  const uint64_t beg[4] = {0, 0, 0, 0};
  return launch_join(sp, 0, sp->hd.n_reads, beg, 0, sp->hd.n, d_out, s);
}

extern "C" int lz_split_scratch_bytes(const lz_split* sp, uint64_t n, uint64_t* bytes) {
  if (!sp || !bytes) return lz_fail(LZ_EINVAL, "lz_split_scratch_bytes: null argument");
  n = std::max<uint64_t>(n, 1);
  uint64_t req = 0, pieces = 0;
  for (int k = 0; k < 4; k++) {
    req = std::max(req, req_scratch(sp, k, n));
    pieces += pad256(n * sp->maxpiece[k]);
  }
  // request tables, request count, piece offsets, pieces, then one stream's request scratch
  *bytes = pad256(4 * n * sizeof(lz_request)) + 256 + pad256(4 * 8 * (n + 1)) + pieces + req;
  return LZ_OK;
}

extern "C" int lz_split_decode_range(lz_split* sp, uint64_t offset, uint64_t len, uint8_t* d_out,
                                     void* d_scratch, uint64_t scratch_len, hipStream_t s) {
  if (!sp || (len && !d_out)) return lz_fail(LZ_EINVAL, "lz_split_decode_range: null argument");
  if (offset > sp->hd.n || len > sp->hd.n - offset) return lz_fail(LZ_ERANGE, "lz_split_decode_range: range outside the file");
  if (!len) return LZ_OK;
  // records covering [offset, offset + len): r0 = last record starting at or
  // before offset, r1 = first record starting at or after the end
  const uint64_t nr = sp->hd.n_reads;
  auto R = [&](uint64_t i) { return sp->hs[i] + 2 * sp->ss[i] + 2 * i; };
  uint64_t lo = 0, hi = nr;                 // largest i < nr with R(i) <= offset
  while (lo < hi) { const uint64_t m = (lo + hi + 1) / 2; if (R(m) <= offset) lo = m; else hi = m - 1; }
  const uint64_t r0 = lo;
  lo = r0; hi = nr;                         // smallest i with R(i) >= offset + len
  while (lo < hi) { const uint64_t m = (lo + hi) / 2; if (R(m) >= offset + len) hi = m; else lo = m + 1; }
  const uint64_t r1 = lo;
  const uint64_t beg[4] = {sp->hs[r0], sp->ss[r0], 2 * r0, sp->ss[r0]};
  const uint64_t end[4] = {sp->hs[r1], sp->ss[r1], 2 * r1, sp->ss[r1]};
  for (int k = 0; k < 4; k++) {
    if (end[k] == beg[k]) continue;
    const int rc = lz_decode_range(sp->sub[k], beg[k], end[k] - beg[k], sp->buf + sp->base[k], d_scratch, scratch_len, s);
    if (rc) return rc;
  }
  return launch_join(sp, r0, r1, beg, offset, offset + len, d_out, s);
}

extern "C" int lz_split_read_lookup(lz_split* sp, const int64_t* d_ids, uint64_t n, uint8_t* d_out,
                                    uint64_t cap, uint64_t* d_offsets, void* d_scratch, uint64_t scratch_len,
                                    hipStream_t s) {
  if (!sp) return lz_fail(LZ_EINVAL, "lz_split_read_lookup: null handle");
  if (!n) return LZ_OK;
  if (!d_ids || !d_out || !d_offsets || !d_scratch) return lz_fail(LZ_EINVAL, "lz_split_read_lookup: null argument");
  if (((uintptr_t)d_scratch & 255)) return lz_fail(LZ_EINVAL, "lz_split_read_lookup: scratch must be 256-byte aligned");
  if (cap < n * (uint64_t)sp->hd.max_rec) return lz_fail(LZ_ECAPACITY, "lz_split_read_lookup: output needs %llu bytes", (unsigned long long)(n * (uint64_t)sp->hd.max_rec));
  uint64_t need = 0;
  lz_split_scratch_bytes(sp, n, &need);
  if (scratch_len < need) return lz_fail(LZ_ECAPACITY, "lz_split_read_lookup: scratch needs %llu bytes", (unsigned long long)need);
  uint8_t* sc = (uint8_t*)d_scratch;
  ReqPlan P{};
  P.hs = sp->d_hs;
  P.ss = sp->d_ss;
  P.ids = d_ids;
  P.n = n;
  P.n_reads = sp->hd.n_reads;
  for (int k = 0; k < 4; k++) P.reqs[k] = reinterpret_cast<lz_request*>(sc) + k * n;
  uint64_t o = pad256(4 * n * sizeof(lz_request));
  P.d_n = reinterpret_cast<uint32_t*>(sc + o);
  o += 256;
  uint64_t* poff[4];
  for (int k = 0; k < 4; k++) poff[k] = reinterpret_cast<uint64_t*>(sc + o) + k * (n + 1);
  o += pad256(4 * 8 * (n + 1));
  uint8_t* piece[4];
  for (int k = 0; k < 4; k++) { piece[k] = sc + o; o += pad256(n * sp->maxpiece[k]); }
  hipLaunchKernelGGL(k_split_reqs, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, P);
  int rc = hip_ok(hipGetLastError(), "k_split_reqs");
  for (int k = 0; k < 4 && !rc; k++)
    rc = lz_decode_batch(sp->sub[k], P.reqs[k], P.d_n, n, piece[k], n * sp->maxpiece[k], poff[k], sc + o,
                         scratch_len - o, s);
  if (rc) return rc;
  GatherArgs G{};
  for (int k = 0; k < 4; k++) { G.piece[k] = piece[k]; G.poff[k] = poff[k]; }
  G.n = n;
  G.out = d_out;
  G.offsets = d_offsets;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((n + 1 + 3) / 4, sp->grid);
  hipLaunchKernelGGL(k_split_gather, dim3(grid), dim3(kJoinWG), 0, s, G);
  return hip_ok(hipGetLastError(), "k_split_gather");
}

extern "C" int lz_split_sync_status(lz_split* sp, hipStream_t s) {
  if (!sp) return lz_fail(LZ_EINVAL, "lz_split_sync_status: null");
  int first = LZ_OK;
  for (auto* h : sp->sub) {
    const int rc = lz_sync_status(h, s);
    if (rc && !first) first = rc;
  }
  return first;
}
