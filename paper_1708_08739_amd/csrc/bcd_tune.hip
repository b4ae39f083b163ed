// Autotuner: measured choice of engine, batch width (column groups), launch
// shape, items per wavefront step and forward direction per graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "../../include/bcd.h"
#include "bcd_host_internal.h"

using namespace bcd;

extern "C" bcd_status bcd_autotune(bcd_graph *gh, bcd_vid r, int32_t max_groups, int64_t max_sources,
                                   bcd_config *best, double *gteps) {
  BCD_GUARD_BEGIN
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
  double best_rate = -1.0;
  bcd_config best_cfg = saved;
  // Times the sample under one configuration: a warm-up batch sizes the
  // workspace, then the timed pass.  *rate < 0 when it could not run
  // (OUT_OF_MEMORY for a batch too wide for the device is not an error).
  auto time_config = [&](const bcd_config &cand, double *rate) -> bcd_status {
    *rate = -1.0;
    STCHK(bcd_set_config(gh, &cand));
    Lease ls(g);
    if (!ls.ok()) return fail(BCD_ERR_OUT_OF_MEMORY, "workspace allocation failed");
    STCHK(ls->init_common(g));
    SourceRun warm, run;
    std::vector<int32_t> head(sample.begin(), sample.begin() + std::min<size_t>(sample.size(), 64));
    bcd_status rc = run_sources(g, ls.w.get(), head, tgt, false, warm);
    if (rc == BCD_ERR_OUT_OF_MEMORY) return BCD_OK;
    STCHK(rc);
    const auto t0 = std::chrono::steady_clock::now();
    rc = run_sources(g, ls.w.get(), sample, tgt, false, run);
    if (rc == BCD_ERR_OUT_OF_MEMORY) return BCD_OK;
    STCHK(rc);
    const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *rate = dt > 0 ? (double)run.te / dt / 1e9 : 0.0;
    if (*rate > best_rate) {
      best_rate = *rate;
      best_cfg = cand;
    }
    return BCD_OK;
  };
  bcd_status rc = BCD_OK;
  // 1. batch width x grid multiplier (block 256, 64 weighted; 2 items per
  //    step, top-down)
  bcd_config cand = saved;
  cand.engine = BCD_ENGINE_BATCHED;
  cand.block = g->weighted ? 64 : 256;
  cand.items = 2;
  cand.bottom_up = 0;
  // widths in powers of two from the largest one <= max_groups / 8 (at
  // least 1) up to max_groups: four widths at most
  int g0 = 1;
  while (g0 * 16 <= max_groups) g0 *= 2;
  for (int G = g0; G <= max_groups && rc == BCD_OK; G *= 2) {
    if ((uint64_t)G * (uint64_t)g->n >= (1ull << 32)) break;
    double widest = -1.0;
    for (int gm : {8, 16, 32}) {
      cand.groups = G;
      cand.grid_mult = gm;
      double rate = -1.0;
      rc = time_config(cand, &rate);
      if (rc != BCD_OK) break;
      widest = std::max(widest, rate);
    }
    if (rc == BCD_OK && widest < 0 && G > 1) break;  // too wide for this device: stop widening
  }
  // 2. around the best: block size; for unweighted graphs also items per
  //    step, bottom-up levels and pushed against pulled path counts
  if (rc == BCD_OK && best_rate >= 0) {
    const bcd_config base = best_cfg;
    std::vector<bcd_config> around;
    bcd_config c = base;
    for (int b : g->weighted ? std::vector<int>{128, 256} : std::vector<int>{512}) {
      c.block = b;
      around.push_back(c);
    }
    if (!g->weighted) {
      for (int it : {1, 4}) {
        c = base;
        c.items = it;
        around.push_back(c);
      }
      for (int bu : {16, 4}) {
        c = base;
        c.bottom_up = bu;
        around.push_back(c);
      }
      c = base;
      c.push = 1 - base.push;
      around.push_back(c);
    }
    for (const bcd_config &x : around) {
      double rate = -1.0;
      rc = time_config(x, &rate);
      if (rc != BCD_OK) break;
    }
  }
  // 3. small unweighted graphs: the LDS engine
  if (rc == BCD_OK && lds_fits(g)) {
    bcd_config c = best_cfg.engine == BCD_ENGINE_BATCHED ? best_cfg : saved;
    c.engine = BCD_ENGINE_LDS;
    double rate = -1.0;
    rc = time_config(c, &rate);
  }
  if (rc != BCD_OK) {
    (void)bcd_set_config(gh, &saved);
    return rc;
  }
  if (best_rate < 0) {
    (void)bcd_set_config(gh, &saved);
    return rc != BCD_OK ? rc : fail(BCD_ERR_DEVICE, "no configuration could be timed");
  }
  (void)bcd_set_config(gh, &best_cfg);
  *best = best_cfg;
  if (gteps) *gteps = best_rate;
  return BCD_OK;
  BCD_GUARD_END
}
