// Checkpoint and resume of an index (svf_save / svf_load): a versioned,
// checksummed little-endian file holding the FP32 vectors, the rows with
// their edge distances, the alive flags, the deletion counters and the
// options that shape results.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "index.hpp"
#include "index_internal.hpp"

namespace {

using svf_detail::fail;

constexpr char kMagic[8] = {'S', 'V', 'F', 'I', 'D', 'X', '0', '1'};
// Version 2 stores localized_repair where version 1 had padding (read as 1).
constexpr int32_t kVersion = 2;

struct FileHeader {
  int32_t version, dim, R, metric;
  int64_t n_slots, n_alive, deleted_since, alive_at_consolidate;
  uint64_t seed;
  int32_t beam_insert, entry_samples, max_iters, search_width, visited_slots, visited_compact,
      repair_c, prune_cap, insert_batch_max, precision, rerank, localized_repair;
  double consolidate_frac;
};

// 64-bit checksum over the bytes of the file in order: FNV-1a's xor-multiply
// step applied to little-endian 8-byte words (a final partial word is
// zero-padded).
class Checksum {
 public:
  void add(const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
      word_ |= (uint64_t)b[i] << (8 * fill_);
      if (++fill_ == 8) flush();
    }
  }
  uint64_t value() {
    if (fill_) flush();
    return h_;
  }

 private:
  void flush() {
    h_ ^= word_;
    h_ *= 0x100000001b3ull;
    word_ = 0;
    fill_ = 0;
  }
  uint64_t h_ = 0xcbf29ce484222325ull, word_ = 0;
  int fill_ = 0;
};

struct File {
  FILE* f = nullptr;
  ~File() {
    if (f) std::fclose(f);
  }
};

bool put(File& fl, Checksum& cs, const void* p, size_t n) {
  cs.add(p, n);
  return std::fwrite(p, 1, n, fl.f) == n;
}
bool get(File& fl, Checksum& cs, void* p, size_t n) {
  if (std::fread(p, 1, n, fl.f) != n) return false;
  cs.add(p, n);
  return true;
}

}  // namespace

extern "C" {

int svf_save(const svf_index* cix, const char* path) {
  if (!cix || !path) return fail(SVF_E_INVAL, "null argument");
  if (cix->server) return fail(SVF_E_BUSY, "index is serving: stop serving first");
  if (cix->bg.active)
    return fail(SVF_E_BUSY, "a background consolidation is pending: call svf_consolidate_wait first");
  svf_index* ix = const_cast<svf_index*>(cix);
  const int64_t n = ix->n_slots;
  FileHeader h{};
  std::vector<float> vecs((size_t)n * ix->dim);
  std::vector<int32_t> rows((size_t)n * ix->R);
  std::vector<float> ed((size_t)n * ix->R);
  std::vector<uint8_t> alive((size_t)n);
  {
    std::lock_guard<std::mutex> g(ix->mu);
    CK(hipStreamSynchronize(ix->stream));
    if (n > 0 && ix->tier.on) {
      // pinned host segments: copied row by row on the host
      for (int64_t i = 0; i < n; ++i)
        std::memcpy(vecs.data() + i * ix->dim, ix->tier.hrow(i, ix->stride), (size_t)ix->dim * 4);
    } else if (n > 0) {
      CK(hipMemcpy2D(vecs.data(), ix->dim * 4, ix->vec32, ix->stride * 4, ix->dim * 4, n,
                     hipMemcpyDefault));
    }
    const svf::Options& o = ix->opt;
    h.version = kVersion;
    h.dim = ix->dim;
    h.R = ix->R;
    h.metric = ix->metric;
    h.n_slots = n;
    h.n_alive = ix->n_alive;
    h.deleted_since = ix->deleted_since;
    h.alive_at_consolidate = ix->alive_at_consolidate;
    h.seed = o.seed;
    h.beam_insert = o.beam_insert;
    h.entry_samples = o.entry_samples;
    h.max_iters = o.max_iters;
    h.search_width = o.search_width;
    h.visited_slots = o.visited_slots;
    h.visited_compact = o.visited_compact;
    h.repair_c = o.repair_c;
    h.prune_cap = o.prune_cap;
    h.insert_batch_max = o.insert_batch_max;
    h.precision = o.precision;
    h.rerank = o.rerank;
    h.consolidate_frac = o.consolidate_frac;
    h.localized_repair = o.localized_repair;
  }
  int rc = svf_export_graph(ix, rows.data(), ed.data(), alive.data(), n);
  if (rc) return rc;
  File fl;
  fl.f = std::fopen(path, "wb");
  if (!fl.f) return fail(SVF_E_INTERNAL, std::string("cannot open for writing: ") + path);
  Checksum cs;
  bool ok = put(fl, cs, kMagic, sizeof kMagic) && put(fl, cs, &h, sizeof h) &&
            put(fl, cs, vecs.data(), vecs.size() * 4) && put(fl, cs, rows.data(), rows.size() * 4) &&
            put(fl, cs, ed.data(), ed.size() * 4) && put(fl, cs, alive.data(), alive.size());
  const uint64_t sum = cs.value();
  ok = ok && std::fwrite(&sum, 1, 8, fl.f) == 8;
  ok = (std::fclose(fl.f) == 0) && ok;
  fl.f = nullptr;
  if (!ok) return fail(SVF_E_INTERNAL, std::string("write failed: ") + path);
  return SVF_OK;
}

int svf_load(const char* path, svf_index** out) {
  if (!path || !out) return fail(SVF_E_INVAL, "null argument");
  *out = nullptr;
  File fl;
  fl.f = std::fopen(path, "rb");
  if (!fl.f) return fail(SVF_E_NOTFOUND, std::string("cannot open: ") + path);
  Checksum cs;
  char magic[8];
  FileHeader h{};
  if (!get(fl, cs, magic, 8) || std::memcmp(magic, kMagic, 8) != 0)
    return fail(SVF_E_INVAL, "not an index file");
  if (!get(fl, cs, &h, sizeof h)) return fail(SVF_E_INVAL, "truncated header");
  if (h.version != kVersion && h.version != 1) return fail(SVF_E_INVAL, "unsupported file version");
  if (h.version == 1) h.localized_repair = 1;
  if (h.dim < 1 || h.dim > 1024 || h.R < 1 || h.R > 128 || h.n_slots < 0 ||
      h.n_slots > (int64_t)INT32_MAX - 64 || h.n_alive < 0 || h.n_alive > h.n_slots)
    return fail(SVF_E_INVAL, "corrupt header");
  const int64_t n = h.n_slots;
  std::vector<float> vecs((size_t)n * h.dim);
  std::vector<int32_t> rows((size_t)n * h.R);
  std::vector<float> ed((size_t)n * h.R);
  std::vector<uint8_t> alive((size_t)n);
  uint64_t sum = 0;
  if (!get(fl, cs, vecs.data(), vecs.size() * 4) || !get(fl, cs, rows.data(), rows.size() * 4) ||
      !get(fl, cs, ed.data(), ed.size() * 4) || !get(fl, cs, alive.data(), alive.size()) ||
      std::fread(&sum, 1, 8, fl.f) != 8)
    return fail(SVF_E_INVAL, "truncated file");
  if (sum != cs.value()) return fail(SVF_E_INVAL, "checksum mismatch");
  svf_index* ix = nullptr;
  int rc = svf_create(h.dim, h.R, h.metric, &ix);
  if (rc) return rc;
  std::unique_ptr<svf_index, int (*)(svf_index*)> guard(ix, svf_destroy);
  ix->opt.seed = h.seed;   // 64 bits: not through the double-valued option call
  const std::pair<const char*, double> opts[] = {
      {"beam_insert", (double)h.beam_insert},
      {"entry_samples", (double)h.entry_samples},
      {"max_iters", (double)h.max_iters},
      {"search_width", (double)h.search_width},
      {"visited_slots", (double)h.visited_slots},
      {"visited_compact", (double)h.visited_compact},
      {"repair_c", (double)h.repair_c},
      {"prune_cap", (double)h.prune_cap},
      {"consolidate_frac", h.consolidate_frac},
      {"insert_batch_max", (double)h.insert_batch_max},
      {"rerank", (double)h.rerank},
      {"localized_repair", (double)h.localized_repair},
  };
  for (const auto& kv : opts) {
    if (kv.first == std::string("beam_insert") && h.beam_insert == 0) continue;   // default
    if ((rc = svf_set_option(ix, kv.first, kv.second))) return rc;
  }
  if ((rc = svf_import_graph(ix, vecs.data(), n, rows.data(), ed.data(), alive.data()))) return rc;
  if (h.precision && (rc = svf_set_option(ix, "precision", (double)h.precision))) return rc;
  ix->deleted_since = h.deleted_since;
  ix->alive_at_consolidate = h.alive_at_consolidate;
  *out = guard.release();
  return SVF_OK;
}

}  // extern "C"
