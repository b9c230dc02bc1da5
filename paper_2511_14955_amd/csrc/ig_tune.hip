// Autotuner for the scan's launch shape: chunk length (symbols per work item),
// workgroup size, and the LDS de-duplication set.  Each candidate runs the
// real pass on the loaded corpus (then the chain is rewound); the fastest
// device pass wins.  Every candidate must return the same table, which the
// tuner checks.  Results can be cached in the file named by IG_TUNE_CACHE,
// keyed by device, corpus shape and pass.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "ig_internal.h"

using namespace ig;

static std::string tune_key(ig_ctx *c, uint32_t n, uint64_t k_keep) {
  hipDeviceProp_t prop{};
  (void)hipGetDeviceProperties(&prop, c->cfg.device);
  char buf[512];
  snprintf(buf, sizeof buf, "%s|cu%d|b%u|f%d|m%llu|s%llu|n%u|k%llu", prop.gcnArchName, c->n_cu, c->cfg.symbol_bits,
           (int)c->cfg.freq, (unsigned long long)c->m, (unsigned long long)c->total_syms, n, (unsigned long long)k_keep);
  for (char *q = buf; *q; q++)
    if (*q == ' ') *q = '_';
  return buf;
}

// A launch shape the scan supports: whole wavefronts per workgroup, a power-of-two LDS set of at
// least one slot per thread (the set's hashing and its flush assume both), chunk length in range.
static bool shape_ok(uint32_t chunk_syms, uint32_t block, uint32_t set_cap) {
  return chunk_syms >= 1024 && chunk_syms <= 65536 && (block == 256 || block == 512 || block == 1024) &&
         set_cap >= 1024 && set_cap <= 32768 && (set_cap & (set_cap - 1)) == 0 && set_cap >= block;
}

// The last line for `key` whose shape is valid (a stale or edited line is ignored).
static bool cache_lookup(const std::string &key, LaunchCfg *lc) {
  const char *path = getenv("IG_TUNE_CACHE");
  if (!path) return false;
  FILE *f = fopen(path, "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  while (fgets(line, sizeof line, f)) {
    char k[600];
    unsigned cs, bl, sc;
    if (sscanf(line, "%599s %u %u %u", k, &cs, &bl, &sc) == 4 && key == k && shape_ok(cs, bl, sc)) {
      lc->chunk_syms = cs;
      lc->block = bl;
      lc->set_cap = sc;
      found = true;
    }
  }
  fclose(f);
  return found;
}

static void cache_store(const std::string &key, const LaunchCfg &lc) {
  const char *path = getenv("IG_TUNE_CACHE");
  if (!path) return;
  FILE *f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s %u %u %u\n", key.c_str(), lc.chunk_syms, lc.block, lc.set_cap);
  fclose(f);
}

extern "C" int ig_autotune(ig_ctx *c, uint32_t n, uint64_t k_keep, ig_tune_report *rep) {
  if (!c) return IG_EINVAL;
  if (c->sticky) return set_error(c, IG_EDEVICE, "context has a sticky device error: %s", c->err.c_str());
  if (c->server) return set_error(c, IG_ESTATE, "serving loop is running");
  if (!c->loaded) return set_error(c, IG_ESTATE, "no corpus loaded");
  if (rep) std::memset(rep, 0, sizeof *rep);
  const std::string key = tune_key(c, n, k_keep);
  const LaunchCfg start = c->lc;
  LaunchCfg cached = start;
  if (cache_lookup(key, &cached)) {
    c->lc = cached;
    if (cached.chunk_syms != start.chunk_syms) {
      int rc = rebuild_chunks(c);
      if (rc) return rc;
    }
    if (rep) {
      rep->n_candidates = 1;
      rep->cand[0].chunk_syms = cached.chunk_syms;
      rep->cand[0].block = cached.block;
      rep->cand[0].set_cap = cached.set_cap;
      rep->cand[0].pass_ms = -1.0;
      rep->best = 0;
      rep->identical = 1;
      rep->from_cache = 1;
    }
    return IG_OK;
  }
  // Chunk lengths are multiples of 1024 symbols (per-thread window runs of chunk / 1024, made
  // odd); 512-thread blocks are kept as a fallback for small corpora, and the largest LDS set
  // only with the shorter chunks.  Shapes that do not fit the pass's LDS are skipped.
  std::vector<LaunchCfg> cands;
  for (uint32_t cs : {15360u, 16384u, 19456u, 23552u, 27648u, 31744u})
    for (uint32_t bl : {512u, 1024u})
      for (uint32_t sc : {4096u, 8192u, 16384u}) {
        if (bl == 512 && cs > 16384) continue;
        if (sc == 16384 && cs > 16384) continue;
        LaunchCfg lc = start;
        lc.chunk_syms = cs;
        lc.block = bl;
        lc.set_cap = sc;
        cands.push_back(lc);
      }
  std::vector<uint64_t> ref_lo, ref_hi, ref_cnt;
  std::vector<ig_key> keys;
  std::vector<uint64_t> counts;
  int best = -1, identical = 1;
  bool have_ref = false;
  double best_ms = 1e30;
  uint32_t cur_chunk = c->lc.chunk_syms;
  for (size_t i = 0; i < cands.size() && i < IG_TUNE_MAX; i++) {
    c->lc = cands[i];
    if (cands[i].chunk_syms != cur_chunk) {
      int rc = rebuild_chunks(c);
      if (rc) return rc;
      cur_chunk = cands[i].chunk_syms;
    }
    double ms = 1e30;
    int ok = 1;
    for (int rep_i = 0; rep_i < 2 && ok; rep_i++) {
      int rc = ig_pass(c, n, k_keep);
      if (rc == IG_EINVAL) { ok = 0; break; }   // launch shape does not fit this pass
      if (rc) return rc;
      ms = std::min(ms, c->last.pass_ms);
      if (rep_i == 0) {
        const uint64_t kept = c->kept;
        keys.resize(kept ? kept : 1);
        counts.resize(kept ? kept : 1);
        uint64_t got = 0;
        rc = ig_topk(c, kept, keys.data(), counts.data(), &got);
        if (rc) return rc;
        if (!have_ref) {
          have_ref = true;
          for (uint64_t j = 0; j < got; j++) {
            ref_lo.push_back(keys[j].lo);
            ref_hi.push_back(keys[j].hi);
            ref_cnt.push_back(counts[j]);
          }
        } else {
          bool same = got == ref_cnt.size();
          for (uint64_t j = 0; same && j < got; j++)
            same = keys[j].lo == ref_lo[j] && keys[j].hi == ref_hi[j] && counts[j] == ref_cnt[j];
          if (!same) identical = 0;
        }
      }
      rc = ig_rewind(c);
      if (rc) return rc;
    }
    if (rep) {
      rep->cand[i].chunk_syms = cands[i].chunk_syms;
      rep->cand[i].block = cands[i].block;
      rep->cand[i].set_cap = cands[i].set_cap;
      rep->cand[i].pass_ms = ok ? ms : -1.0;
      rep->n_candidates = (uint32_t)(i + 1);
    }
    if (!ok) continue;
    if (ms < best_ms) {
      best_ms = ms;
      best = (int)i;
    }
  }
  if (best < 0) {
    c->lc = start;
    if (cur_chunk != start.chunk_syms) (void)rebuild_chunks(c);
    return set_error(c, IG_EINVAL, "no launch shape fits this pass");
  }
  c->lc = cands[best];
  if (cur_chunk != cands[best].chunk_syms) {
    int rc = rebuild_chunks(c);
    if (rc) return rc;
  }
  if (rep) {
    rep->best = (uint32_t)best;
    rep->identical = identical;
  }
  if (!identical) return set_error(c, IG_EDEVICE, "launch shapes gave different tables");
  cache_store(key, c->lc);
  return IG_OK;
}

extern "C" int ig_get_launch(const ig_ctx *c, uint32_t *chunk_syms, uint32_t *block, uint32_t *set_cap) {
  if (!c) return IG_EINVAL;
  if (chunk_syms) *chunk_syms = c->lc.chunk_syms;
  if (block) *block = c->lc.block;
  if (set_cap) *set_cap = c->lc.set_cap;
  return IG_OK;
}

extern "C" int ig_set_launch(ig_ctx *c, uint32_t chunk_syms, uint32_t block, uint32_t set_cap) {
  if (!c) return IG_EINVAL;
  if (c->server) return set_error(c, IG_ESTATE, "serving loop is running");
  if (!shape_ok(chunk_syms, block, set_cap)) return set_error(c, IG_EINVAL, "bad launch shape");
  const bool rechunk = chunk_syms != c->lc.chunk_syms;
  c->lc.chunk_syms = chunk_syms;
  c->lc.block = block;
  c->lc.set_cap = set_cap;
  if (rechunk && c->loaded) return rebuild_chunks(c);
  return IG_OK;
}
