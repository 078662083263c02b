// Test driver of the CPU emulation: decode an archive through the C ABI
// (whole file, three ranges, and four reads when it has a read index) and
// compare every byte with the source.  Prints "emu ok" and exits 0 on success.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "lz.h"

static std::vector<uint8_t> slurp(const char* p) {
  std::vector<uint8_t> v;
  FILE* f = std::fopen(p, "rb");
  if (!f) { std::perror(p); std::exit(2); }
  uint8_t buf[1 << 16];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) v.insert(v.end(), buf, buf + n);
  std::fclose(f);
  return v;
}

static uint8_t* aligned(size_t n) {
  void* p = nullptr;
  if (posix_memalign(&p, 256, n ? n : 1)) std::exit(3);
  std::memset(p, 0xAA, n ? n : 1);
  return (uint8_t*)p;
}

#define CHECK(x) do { int rc_ = (x); if (rc_) { std::fprintf(stderr, "%s -> %d: %s\n", #x, rc_, lz_last_error()); return 1; } } while (0)

int main(int argc, char** argv) {
  if (argc < 3) { std::fprintf(stderr, "usage: emu archive source\n"); return 2; }
  std::vector<uint8_t> av = slurp(argv[1]), src = slurp(argv[2]);
  uint8_t* arc = aligned(av.size());
  std::memcpy(arc, av.data(), av.size());
  lz_info info;
  CHECK(lz_info_get(arc, av.size(), &info));
  if (info.n != src.size()) { std::fprintf(stderr, "size mismatch\n"); return 1; }
  uint8_t* ws = aligned(info.workspace_bytes);
  lz_handle* h = nullptr;
  CHECK(lz_open(arc, av.size(), ws, info.workspace_bytes, nullptr, &h));
  const uint64_t N = info.n, B = 1ull << info.block_log2;
  uint8_t* out = aligned(N + 256);
  CHECK(lz_decode_all(h, out, N + 256, nullptr));
  CHECK(lz_sync_status(h, nullptr));
  if (std::memcmp(out, src.data(), N)) { std::fprintf(stderr, "whole-file decode differs\n"); return 1; }
  // ranges
  const uint64_t scr_len = 256 + 64 * 1024 + info.n_blocks * B;
  uint8_t* scr = aligned(scr_len);
  const uint64_t offs[3] = {0, N / 3, N > 5000 ? N - 5000 : 0};
  const uint64_t lens[3] = {N < 3000 ? N : 3000, N / 3 < 7777 ? N / 3 : 7777, N < 5000 ? N : 5000};
  for (int k = 0; k < 3; k++) {
    uint8_t* r = aligned(lens[k] + 256);
    std::memset(scr, 0xAA, scr_len);
    CHECK(lz_decode_range(h, offs[k], lens[k], r, scr, scr_len, nullptr));
    CHECK(lz_sync_status(h, nullptr));
    if (std::memcmp(r, src.data() + offs[k], lens[k])) { std::fprintf(stderr, "range %d differs\n", k); return 1; }
    std::free(r);
  }
  // reads (records of four lines)
  if (info.n_reads) {
    std::vector<uint64_t> rs{0};
    int lines = 0;
    for (uint64_t i = 0; i < N; i++)
      if (src[i] == '\n' && ++lines % 4 == 0) rs.push_back(i + 1);
    const int64_t ids_h[4] = {0, (int64_t)info.n_reads - 1, (int64_t)info.n_reads / 2, (int64_t)info.n_reads / 2};
    int64_t* ids = (int64_t*)aligned(sizeof(ids_h));
    std::memcpy(ids, ids_h, sizeof(ids_h));
    uint64_t* offsets = (uint64_t*)aligned(8 * 5);
    const uint64_t cap = 4 * (uint64_t)info.max_record_len;
    uint8_t* r = aligned(cap);
    std::memset(scr, 0xAA, scr_len);
    CHECK(lz_read_lookup(h, ids, 4, r, cap, offsets, scr, scr_len, nullptr));
    CHECK(lz_sync_status(h, nullptr));
    for (int k = 0; k < 4; k++) {
      const uint64_t a = rs[ids_h[k]], b = rs[ids_h[k] + 1];
      if (offsets[k + 1] - offsets[k] != b - a || std::memcmp(r + offsets[k], src.data() + a, b - a)) {
        std::fprintf(stderr, "read %d differs\n", k);
        return 1;
      }
    }
    std::free(ids);
    std::free(offsets);
    std::free(r);
  }
  // the eight-kernel request path (planning in one workgroup switched off)
  lz_tuning tu;
  CHECK(lz_get_tuning(h, &tu));
  tu.plan_blocks = 1;
  CHECK(lz_set_tuning(h, &tu));
  for (int k = 0; k < 3; k++) {
    uint8_t* r = aligned(lens[k] + 256);
    std::memset(scr, 0xAA, scr_len);
    CHECK(lz_decode_range(h, offs[k], lens[k], r, scr, scr_len, nullptr));
    CHECK(lz_sync_status(h, nullptr));
    if (std::memcmp(r, src.data() + offs[k], lens[k])) { std::fprintf(stderr, "range %d differs (8 kernels)\n", k); return 1; }
    std::free(r);
  }
  // a batch of two ranges (and two reads when there is a read index)
  {
    const int nreq = info.n_reads ? 4 : 2;
    lz_request* rq = (lz_request*)aligned(sizeof(lz_request) * 4);
    rq[0] = lz_request{1, (int64_t)(N / 5), (int64_t)(N / 5 < 1000 ? N / 5 : 1000)};
    rq[1] = lz_request{1, 0, (int64_t)(N < 700 ? N : 700)};
    if (info.n_reads) {
      rq[2] = lz_request{0, 0, 0};
      rq[3] = lz_request{0, (int64_t)info.n_reads - 1, 0};
    }
    uint32_t* dn = (uint32_t*)aligned(4);
    *dn = (uint32_t)nreq;
    uint64_t* offsets = (uint64_t*)aligned(8 * 5);
    const uint64_t cap = 2000 + 2 * (uint64_t)info.max_record_len;
    uint8_t* r = aligned(cap);
    for (uint32_t pb : {4096u, 1u}) {
      tu.plan_blocks = pb;
      CHECK(lz_set_tuning(h, &tu));
      std::memset(scr, 0xAA, scr_len);
      CHECK(lz_decode_batch(h, rq, dn, nreq, r, cap, offsets, scr, scr_len, nullptr));
      CHECK(lz_sync_status(h, nullptr));
      std::vector<uint8_t> want;
      for (int k = 0; k < nreq; k++) {
        uint64_t a0 = (uint64_t)rq[k].a, b0 = a0 + (uint64_t)rq[k].b;
        if (rq[k].kind == 0) {
          std::vector<uint64_t> rs{0};
          int lines = 0;
          for (uint64_t i = 0; i < N; i++)
            if (src[i] == '\n' && ++lines % 4 == 0) rs.push_back(i + 1);
          a0 = rs[rq[k].a];
          b0 = rs[rq[k].a + 1];
        }
        want.insert(want.end(), src.begin() + a0, src.begin() + b0);
      }
      if (offsets[nreq] != want.size() || std::memcmp(r, want.data(), want.size())) {
        std::fprintf(stderr, "batch differs (plan_blocks %u)\n", pb);
        return 1;
      }
    }
    std::free(rq);
    std::free(dn);
    std::free(offsets);
    std::free(r);
  }
  // device verification hash
  {
    uint64_t* tree = (uint64_t*)aligned(8);
    uint8_t* vs = aligned(8 * info.n_blocks + 8);
    CHECK(lz_verify(h, out, tree, vs, 8 * info.n_blocks + 8, nullptr));
    CHECK(lz_sync_status(h, nullptr));
    if (*tree != info.source_fnv) { std::fprintf(stderr, "verification tree differs\n"); return 1; }
    std::free(tree);
    std::free(vs);
  }
  lz_close(h);
  std::free(arc);
  std::free(ws);
  std::free(out);
  std::free(scr);
  std::printf("emu ok: %llu bytes, %llu blocks\n", (unsigned long long)N, (unsigned long long)info.n_blocks);
  return 0;
}
