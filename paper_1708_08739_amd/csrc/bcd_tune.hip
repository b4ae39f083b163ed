// Autotuner for the batched engine: measured choice of batch width
// (column groups) and launch shape per graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "../../include/bcd.h"
#include "bcd_host_internal.h"

using namespace bcd;

extern "C" bcd_status bcd_autotune(bcd_graph *gh, bcd_vid r, int32_t max_groups, int64_t max_sources,
                                   bcd_config *best, double *gteps) {
  if (!gh || !best || max_groups < 1 || max_sources < 1) return fail(BCD_ERR_INVALID_ARG, "bad argument");
  Graph *g = reinterpret_cast<Graph *>(gh);
  if (r < 0 || r >= g->n) return fail(BCD_ERR_INVALID_ARG, "r out of range");
  const bcd_config saved = g->config();
  std::vector<int32_t> rv;
  {
    Lease ls(g);
    if (!ls.ok()) return fail(BCD_ERR_OUT_OF_MEMORY, "workspace allocation failed");
    STCHK(ls->init_common(g));
    std::vector<uint32_t> bits;
    int64_t k = 0;
    STCHK(reach_set(g, ls.w.get(), r, true, bits, &k, nullptr));
    bits_to_list(bits, g->n, r, rv);
  }
  if (rv.empty()) return fail(BCD_ERR_INVALID_ARG, "RV(r) is empty");
  // seeded, spread-out sample of RV(r)
  std::vector<int32_t> sample;
  const size_t want = (size_t)std::min<int64_t>(max_sources, (int64_t)rv.size());
  for (size_t i = 0; i < want; ++i) sample.push_back(rv[(size_t)(index_below(splitmix_at(0x5EEDull, i), rv.size()))]);
  std::sort(sample.begin(), sample.end());
  sample.erase(std::unique(sample.begin(), sample.end()), sample.end());
  std::vector<int32_t> tgt{r};
  bcd_config cand = saved;
  cand.engine = BCD_ENGINE_BATCHED;
  double best_rate = -1.0;
  bcd_config best_cfg = saved;
  bcd_status rc = BCD_OK;
  for (int G = 1; G <= max_groups && rc == BCD_OK; G *= 2) {
    if ((uint64_t)G * (uint64_t)g->n >= (1ull << 32)) break;
    for (int block : {256, 512}) {
      for (int gm : {8, 16, 32}) {
        cand.groups = G;
        cand.block = block;
        cand.grid_mult = gm;
        rc = bcd_set_config(gh, &cand);
        if (rc != BCD_OK) break;
        Lease ls(g);
        if (!ls.ok()) {
          rc = fail(BCD_ERR_OUT_OF_MEMORY, "workspace allocation failed");
          break;
        }
        rc = ls->init_common(g);
        if (rc != BCD_OK) break;
        SourceRun warm, run;
        // one warm-up batch sizes the workspace, then the timed pass
        std::vector<int32_t> head(sample.begin(), sample.begin() + std::min<size_t>(sample.size(), 64));
        rc = run_sources(g, ls.w.get(), head, tgt, false, warm);
        if (rc == BCD_OK) {
          const auto t0 = std::chrono::steady_clock::now();
          rc = run_sources(g, ls.w.get(), sample, tgt, false, run);
          const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
          const double rate = dt > 0 ? (double)run.te / dt / 1e9 : 0.0;
          if (rc == BCD_OK && rate > best_rate) {
            best_rate = rate;
            best_cfg = cand;
          }
        }
        if (rc == BCD_ERR_OUT_OF_MEMORY && G > 1) {  // too wide for this device: stop widening
          rc = BCD_OK;
          G = max_groups;
          break;
        }
        if (rc != BCD_OK) break;
      }
      if (rc != BCD_OK) break;
    }
  }
  if (best_rate < 0) {
    (void)bcd_set_config(gh, &saved);
    return rc != BCD_OK ? rc : fail(BCD_ERR_DEVICE, "no configuration could be timed");
  }
  (void)bcd_set_config(gh, &best_cfg);
  *best = best_cfg;
  if (gteps) *gteps = best_rate;
  return BCD_OK;
}
