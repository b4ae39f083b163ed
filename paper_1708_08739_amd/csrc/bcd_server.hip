// libbcd serving loop: many BC(r) queries on one resident graph with
// continuous batching at source granularity.
//
// Threads:
//   planner  - takes submitted queries in arrival order, finds RV(r) (or the
//              union D for a set query, or the draws of Alg.2), reserves the
//              query's device result buffer against the HBM budget (waiting
//              while it does not fit) and publishes its source list;
//   workers  - each owns a batch workspace and a stream; a worker fills its
//              next batch with the next unscheduled sources of the admitted
//              queries in admission order (one lane per distinct vertex: a
//              source two queries need is computed once), runs the batched
//              pass, and routes each lane's dependency on each of its
//              queries' targets straight into those queries' device buffers;
//   the worker that completes a query's last source copies its buffer back,
//   reduces it exactly as the standalone call does, and posts the result.
// A query that arrives while batches run is admitted as budget frees up and
// joins the following batches, so its work overlaps with the others on the
// device; its value is bit-identical to the standalone call (per-source
// dependencies do not depend on batch composition, and the reduction order
// is the same).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/bcd.h"
#include "bcd_host_internal.h"

namespace bcd {

static double steady_now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct SQuery {
  uint64_t ticket = 0;
  bcd_query q{};
  std::vector<int32_t> rs;       // set targets as submitted
  std::vector<int32_t> targets;  // distinct targets
  std::vector<int32_t> sources;  // distinct sources, in reduction order
  std::vector<int64_t> draw;     // sampled: draw -> source slot
  std::vector<uint32_t> order;   // scheduling order of the source slots
  double *dres = nullptr;        // device [ns][nt]
  size_t bytes = 0;
  size_t next = 0;               // next source to schedule
  size_t done = 0;               // sources finished
  bool overflow = false;
  bool failed = false;
  bcd_result res{};
};

}  // namespace bcd

struct bcd_server {
  bcd::Graph *g = nullptr;
  bcd_server_config cfg{};
  std::mutex mu;
  std::condition_variable cv_plan;     // planner: new submissions / budget freed / stop
  std::condition_variable cv_work;     // workers: admitted work / stop
  std::condition_variable cv_done;     // pollers
  std::condition_variable cv_drained;  // shutdown: planner idle and nothing admitted
  std::deque<std::shared_ptr<bcd::SQuery>> submitted;
  std::deque<std::shared_ptr<bcd::SQuery>> active;  // admitted, in admission order
  std::deque<bcd_result> finished;
  size_t outstanding = 0;  // submitted and not yet polled
  size_t reserved = 0;     // bytes of the buffers admitted queries hold
  // device result buffers of finished queries, kept for reuse by size (a
  // free in the serving loop would wait for every stream of the device);
  // reserved + cached never exceeds budget_q
  std::multimap<size_t, double *> cache;
  size_t cached = 0;
  size_t budget_q = 0;     // budget left for query buffers after workspaces
  uint64_t next_ticket = 1;
  bool stop = false;
  bool closing = false;    // shutdown: no new submissions, nothing more admitted
  bool planning = false;   // the planner holds a query it took from `submitted`
  std::thread planner;
  std::vector<std::thread> workers;
  std::vector<std::unique_ptr<bcd::Workspace>> wss;
  std::unique_ptr<bcd::Workspace> plan_ws;
  bcd_server_stats stats{};
};

namespace bcd {

static void post_result(bcd_server *S, const std::shared_ptr<SQuery> &q, int32_t status) {
  q->res.status = status;
  q->res.t_done_s = steady_now();
  S->finished.push_back(q->res);
  S->cv_done.notify_all();
}

// Reduce a finished query exactly as the standalone calls do.
static bcd_status finalize(bcd_server *S, Workspace *ws, SQuery &q) {
  const size_t ns = q.sources.size(), nt = q.targets.size();
  std::vector<double> dep(ns * nt);
  if (ns * nt > 0) {
    if (hipMemcpyAsync(dep.data(), q.dres, ns * nt * sizeof(double), hipMemcpyDeviceToHost, ws->stream) !=
            hipSuccess ||
        hipStreamSynchronize(ws->stream) != hipSuccess)
      return fail(BCD_ERR_DEVICE, "result copy failed");
  }
  Graph *g = S->g;
  if (q.q.kind == BCD_QUERY_EXACT) {
    q.res.bc = compensated_sum(dep.data(), ns, 1);
  } else if (q.q.kind == BCD_QUERY_SAMPLED) {
    if (q.res.stats.ran_exact) {
      q.res.bc = compensated_sum(dep.data(), ns, 1);
    } else {
      std::vector<double> seq(q.draw.size());
      for (size_t t = 0; t < q.draw.size(); ++t) seq[t] = dep[(size_t)q.draw[t]];
      q.res.bc = compensated_sum(seq.data(), seq.size(), 1) * (double)q.res.stats.rv_size / (double)seq.size();
    }
  } else {
    for (size_t i = 0; i < q.rs.size(); ++i) {
      const size_t t = (size_t)(std::lower_bound(q.targets.begin(), q.targets.end(), q.rs[i]) - q.targets.begin());
      const double v = g->outdeg(q.rs[i]) == 0 ? 0.0 : compensated_sum(dep.data() + t, ns, nt);
      q.q.bc_out[i] = v;
      if (i == 0) q.res.bc = v;
    }
  }
  return BCD_OK;
}

// Source list of a query (same rules as bcd_bc_exact / _sampled / _set).
static bcd_status plan_query(bcd_server *S, Workspace *ws, SQuery &q) {
  Graph *g = S->g;
  bcd_stats &st = q.res.stats;
  st.fr_size = -1;
  std::vector<uint32_t> bits;
  int64_t k = 0;
  if (q.q.kind == BCD_QUERY_SET) {
    q.targets = q.rs;
    std::sort(q.targets.begin(), q.targets.end());
    q.targets.erase(std::unique(q.targets.begin(), q.targets.end()), q.targets.end());
    std::vector<uint32_t> uni((size_t)(g->n + 31) / 32, 0u);
    for (int32_t r : q.targets) {
      if (g->outdeg(r) == 0) continue;
      STCHK(reach_set(g, ws, r, true, bits, &k, nullptr));
      bits[(size_t)r >> 5] &= ~(1u << (r & 31));
      for (size_t i = 0; i < uni.size(); ++i) uni[i] |= bits[i];
    }
    bits_to_list(uni, g->n, -1, q.sources);
    st.rv_size = (int64_t)q.sources.size();
    st.distinct_sources = st.rv_size;
    return BCD_OK;
  }
  const int32_t r = q.q.r;
  q.targets = {r};
  if (g->outdeg(r) == 0) {
    st.rv_size = -1;
    return BCD_OK;
  }
  const bcd_sample_params &p = q.q.params;
  // the unpruned baseline of bcd_bc_sampled: every vertex but r is a
  // candidate source, with n - 1 in Eq.(8) and no exact fallback
  const bool all_v = q.q.kind == BCD_QUERY_SAMPLED && (p.flags & BCD_SAMPLE_ALL_VERTICES) != 0;
  std::vector<int32_t> rv;
  if (all_v) {
    rv.reserve((size_t)g->n - 1);
    for (int64_t v = 0; v < g->n; ++v)
      if (v != r) rv.push_back((int32_t)v);
    k = (int64_t)rv.size();
  } else {
    STCHK(reach_set(g, ws, r, true, bits, &k, nullptr));
    bits_to_list(bits, g->n, r, rv);
  }
  st.rv_size = k;
  if (q.q.kind == BCD_QUERY_EXACT) {
    q.sources = std::move(rv);
    st.distinct_sources = (int64_t)q.sources.size();
    return BCD_OK;
  }
  int64_t T = p.T_override;
  if (T <= 0) {
    double K = (double)(g->n - 2);
    if (!(p.flags & BCD_K_TRIVIAL)) {
      int64_t fr = 0;
      std::vector<uint32_t> fb;
      STCHK(reach_set(g, ws, r, false, fb, &fr, nullptr));
      st.fr_size = fr;
      K = (double)fr;
    }
    const double eps_abs = (p.flags & BCD_EPS_ABSOLUTE) ? p.eps : p.eps * (double)g->n * (double)(g->n - 1);
    STCHK(bcd_sample_count(eps_abs, p.delta, K, k, &T));
  }
  st.samples = T;
  if (k == 0) return BCD_OK;
  if (T >= k && !(p.flags & (BCD_NO_EXACT_FALLBACK | BCD_SAMPLE_ALL_VERTICES))) {
    st.ran_exact = 1;
    q.sources = std::move(rv);
  } else {
    if (T > (int64_t)1 << 40) return fail(BCD_ERR_UNSUPPORTED, "sample count too large to draw");
    std::vector<int64_t> slot((size_t)k, -1);
    q.draw.resize((size_t)T);
    for (int64_t t = 0; t < T; ++t) {
      const uint64_t idx = index_below(splitmix_at(p.seed, (uint64_t)t), (uint64_t)k);
      if (slot[idx] < 0) {
        slot[idx] = (int64_t)q.sources.size();
        q.sources.push_back(rv[idx]);
      }
      q.draw[(size_t)t] = slot[idx];
    }
  }
  st.distinct_sources = (int64_t)q.sources.size();
  return BCD_OK;
}

// The planner has disposed of the query it took (posted or admitted); called
// with the server lock held.
static void plan_done(bcd_server *S) {
  S->planning = false;
  S->cv_drained.notify_all();
}

static void planner_loop(bcd_server *S) {
  Workspace *ws = S->plan_ws.get();
  for (;;) {
    std::shared_ptr<SQuery> q;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_plan.wait(lk, [&] { return S->stop || !S->submitted.empty(); });
      if (S->stop) return;
      q = S->submitted.front();
      S->submitted.pop_front();
      S->planning = true;
    }
    const double t0 = steady_now();
    bcd_status rc = BCD_OK;
    try {
      rc = plan_query(S, ws, *q);
      if (rc == BCD_OK) rc = source_order(S->g, ws, q->sources, q->order);
    } catch (const std::bad_alloc &) {
      rc = fail(BCD_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
      rc = fail(BCD_ERR_DEVICE, "unexpected host exception");
    }
    q->res.stats.t_rv_s = steady_now() - t0;
    const size_t cells = q->sources.size() * q->targets.size();
    q->bytes = std::max<size_t>(cells, 1) * sizeof(double);
    std::unique_lock<std::mutex> lk(S->mu);
    if (rc != BCD_OK) {
      post_result(S, q, rc);
      plan_done(S);
      continue;
    }
    if (S->closing) {
      post_result(S, q, BCD_ERR_CANCELLED);
      plan_done(S);
      continue;
    }
    if (cells == 0) {  // nothing to compute (out-degree 0, empty RV)
      q->res.t_admit_s = steady_now();
      q->res.bc = 0.0;
      if (q->q.kind == BCD_QUERY_SET)
        for (size_t i = 0; i < q->rs.size(); ++i) q->q.bc_out[i] = 0.0;
      post_result(S, q, BCD_OK);
      plan_done(S);
      continue;
    }
    if (q->bytes > S->budget_q) {
      lk.unlock();
      fail(BCD_ERR_OUT_OF_MEMORY, "query result buffer exceeds the server's HBM budget");
      lk.lock();
      post_result(S, q, BCD_ERR_OUT_OF_MEMORY);
      plan_done(S);
      continue;
    }
    // admission: wait until the buffer fits the budget
    S->cv_plan.wait(lk, [&] { return S->stop || S->closing || S->reserved + q->bytes <= S->budget_q; });
    if (S->stop || S->closing) {
      post_result(S, q, BCD_ERR_CANCELLED);
      plan_done(S);
      if (S->stop) return;
      continue;
    }
    // a cached buffer of fitting size (at most twice the need), else a new
    // one once the cache has given back what the budget needs
    const size_t need = q->bytes;
    std::vector<double *> trim;
    auto it = S->cache.lower_bound(need);
    if (it != S->cache.end() && it->first <= 2 * need && S->reserved + it->first <= S->budget_q) {
      q->dres = it->second;
      q->bytes = it->first;
      S->cached -= it->first;
      S->cache.erase(it);
    } else {
      while (!S->cache.empty() && S->reserved + S->cached + need > S->budget_q) {
        auto last = std::prev(S->cache.end());
        trim.push_back(last->second);
        S->cached -= last->first;
        S->cache.erase(last);
      }
    }
    S->reserved += q->bytes;
    lk.unlock();
    for (double *p : trim) (void)hipFree(p);
    bcd_status arc = BCD_OK;
    if (!q->dres && hipMalloc((void **)&q->dres, q->bytes) != hipSuccess) {
      (void)hipGetLastError();
      q->dres = nullptr;
      arc = BCD_ERR_OUT_OF_MEMORY;
    } else if (hipMemsetAsync(q->dres, 0, need, ws->stream) != hipSuccess ||
               hipStreamSynchronize(ws->stream) != hipSuccess) {
      arc = BCD_ERR_DEVICE;
    }
    lk.lock();
    if (arc != BCD_OK) {
      S->reserved -= q->bytes;
      if (q->dres) {
        S->cache.emplace(q->bytes, q->dres);
        S->cached += q->bytes;
      }
      q->dres = nullptr;
      post_result(S, q, arc);
      plan_done(S);
      continue;
    }
    q->res.t_admit_s = steady_now();
    S->active.push_back(q);
    S->cv_work.notify_all();
    plan_done(S);
  }
}

struct Lane {
  int32_t vertex;
  std::vector<std::pair<std::shared_ptr<SQuery>, uint32_t>> users;  // (query, source slot)
};

// Called with the server lock held: the buffer goes back to the cache.
static void release_query(bcd_server *S, SQuery &q) {
  if (q.dres) {
    S->cache.emplace(q.bytes, q.dres);
    S->cached += q.bytes;
  }
  q.dres = nullptr;
  S->reserved -= q.bytes;
  S->cv_plan.notify_all();
}

static void worker_loop(bcd_server *S, Workspace *ws) {
  Graph *g = S->g;
  const size_t width = (size_t)ws->G * kLanes;
  std::vector<unsigned long long> ovl((size_t)ws->G);
  for (;;) {
    std::vector<Lane> lanes;
    std::vector<int32_t> tg;  // distinct targets of the batch
    bcd_status rc = BCD_OK;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] {
        if (S->stop) return true;
        for (auto &q : S->active)
          if (q->next < q->sources.size()) return true;
        return false;
      });
      if (S->stop) return;
      // an exception here (host allocation) fails the lanes taken so far
      try {
        std::unordered_map<int32_t, size_t> where;
        for (auto &q : S->active) {
          while (q->next < q->sources.size() && lanes.size() < width) {
            const uint32_t slot = q->order[q->next];
            const int32_t s = q->sources[slot];
            auto it = where.find(s);
            if (it == where.end()) {
              where.emplace(s, lanes.size());
              lanes.push_back(Lane{s, {}});
              it = where.find(s);
            }
            lanes[it->second].users.emplace_back(q, slot);
            q->next++;
          }
          if (lanes.size() >= width) break;
        }
        for (auto &ln : lanes)
          for (auto &u : ln.users)
            for (int32_t t : u.first->targets) tg.push_back(t);
      } catch (const std::bad_alloc &) {
        rc = BCD_ERR_OUT_OF_MEMORY;
      } catch (...) {
        rc = BCD_ERR_DEVICE;
      }
    }
    const int k = (int)lanes.size();
    int32_t *d_t = nullptr;
    ResultRoute *d_routes = nullptr;
    ProfAcc prof;
    bool ovf = false;
    uint64_t ctr[C_COUNT] = {0};
    int ntgt = 0;
    bool threw = false;
    try {
      // an earlier batch whose item-list growth failed left this workspace to
      // be rebuilt (both calls return at once when it is ready)
      if (rc == BCD_OK) rc = ws->ensure_batch(S->cfg.groups);
      if (rc == BCD_OK && g->weighted) rc = ws->ensure_weighted();
      if (rc == BCD_OK) {
        std::sort(tg.begin(), tg.end());
        tg.erase(std::unique(tg.begin(), tg.end()), tg.end());
        // stage the batch
        {
          std::vector<int32_t> bsrc((size_t)k);
          for (int i = 0; i < k; ++i) bsrc[(size_t)i] = lanes[(size_t)i].vertex;
          ws->stage_sources(bsrc.data(), k);
        }
        ntgt = (int)tg.size();
        rc = ws->ensure_res((size_t)std::max(ntgt, 1) * width);
        std::vector<ResultRoute> routes;
        for (int i = 0; i < k; ++i)
          for (auto &u : lanes[(size_t)i].users) {
            SQuery &q = *u.first;
            const size_t nt = q.targets.size();
            for (size_t ti = 0; ti < nt; ++ti) {
              const size_t t = (size_t)(std::lower_bound(tg.begin(), tg.end(), q.targets[ti]) - tg.begin());
              ResultRoute rr;
              rr.dst = q.dres + (size_t)u.second * nt + ti;
              rr.src = (uint32_t)(t * width + (size_t)i);
              rr.pad = 0;
              routes.push_back(rr);
            }
          }
        if (rc == BCD_OK) rc = ws->ensure_server_lists((size_t)ntgt, routes.size());
        if (rc == BCD_OK) {
          d_t = ws->d_tgt_list;
          d_routes = ws->d_routes;
          hipError_t e = hipMemcpyAsync(d_t, tg.data(), (size_t)ntgt * sizeof(int32_t), hipMemcpyHostToDevice, ws->stream);
          if (e == hipSuccess)
            e = hipMemcpyAsync(d_routes, routes.data(), routes.size() * sizeof(ResultRoute), hipMemcpyHostToDevice,
                               ws->stream);
          if (e == hipSuccess) e = launch_scatter_targets(ws->S.tgt_of, d_t, ntgt, 1, ws->stream);
          if (e != hipSuccess) rc = BCD_ERR_DEVICE;
        }
        if (rc == BCD_OK) rc = run_staged_batch(g, ws, k, ntgt, ovl.data(), &ovf, &prof);
        if (rc == BCD_OK) {
          hipError_t e = launch_route_results(ws->S.res, d_routes, (int)routes.size(), ws->stream);
          if (e == hipSuccess) e = hipStreamSynchronize(ws->stream);
          if (e != hipSuccess) rc = BCD_ERR_DEVICE;
        }
        if (d_t) {
          (void)launch_scatter_targets(ws->S.tgt_of, d_t, ntgt, 0, ws->stream);
          (void)hipStreamSynchronize(ws->stream);
        }
        d_t = nullptr;
        d_routes = nullptr;
        if (rc == BCD_OK) rc = collect_counters(ws, ctr, ws->S.acc);
        if (rc == BCD_OK && g->profiling.load()) record_profile(g, prof, ctr);
      }
    } catch (const std::bad_alloc &) {
      rc = BCD_ERR_OUT_OF_MEMORY;
      threw = true;
    } catch (...) {
      rc = BCD_ERR_DEVICE;
      threw = true;
    }
    if (threw) {  // leave the workspace as a finished batch would
      (void)hipStreamSynchronize(ws->stream);
      if (d_t) (void)launch_scatter_targets(ws->S.tgt_of, d_t, ntgt, 0, ws->stream);
      (void)ws->reset_batch_dense();
      (void)hipStreamSynchronize(ws->stream);
    }
    // account
    std::vector<std::shared_ptr<SQuery>> complete;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->stats.batches += 1;
      S->stats.lanes_used += (uint64_t)k;
      S->stats.lane_slots += (uint64_t)width;
      S->stats.traversed_edges += ctr[C_FWD_APAIRS];
      for (auto &ln : lanes)
        if (ln.users.size() > 1) S->stats.shared_lanes += 1;
      for (int i = 0; i < k; ++i) {
        const bool lane_ovf = ovf && ((ovl[(size_t)i / kLanes] >> (i % kLanes)) & 1ull);
        for (auto &u : lanes[(size_t)i].users) {
          SQuery &q = *u.first;
          if (rc != BCD_OK) q.failed = true;
          if (lane_ovf) q.overflow = true;
          q.done++;
          if (q.done == q.sources.size()) complete.push_back(u.first);
        }
      }
      // a query whose every source has been counted leaves the active list
      for (auto &q : complete) {
        auto it = std::find(S->active.begin(), S->active.end(), q);
        if (it != S->active.end()) S->active.erase(it);
      }
    }
    for (auto &q : complete) {
      int32_t status = BCD_OK;
      if (q->failed) status = rc != BCD_OK ? rc : BCD_ERR_DEVICE;
      else if (q->overflow) status = BCD_ERR_SIGMA_OVERFLOW;
      else {
        bcd_status fr = finalize(S, ws, *q);
        if (fr != BCD_OK) status = fr;
      }
      q->res.stats.t_bc_s = steady_now() - q->res.t_admit_s;
      q->res.stats.batch_width = (int32_t)width;
      std::unique_lock<std::mutex> lk(S->mu);
      release_query(S, *q);
      S->stats.queries_done += 1;
      post_result(S, q, status);
      S->cv_drained.notify_all();
    }
  }
}

}  // namespace bcd

using namespace bcd;

namespace bcd {

// Device bytes of one worker's batch workspace of `groups` column groups:
// 64-bit path-count and psi rows, backward level masks, initial item lists
// of 16 entries per (g, v), the per-vertex target map, and the engine's own
// arrays (weighted: distances, DAG in-arc counters, round masks, per-arc DAG
// lane masks; unweighted: level records).
uint64_t batch_workspace_bytes(const Graph *g, int groups) {
  const uint64_t GN = (uint64_t)groups * (uint64_t)g->n;
  uint64_t b = GN * kLanes * 16 + GN * 2 * sizeof(LevMask) + GN * 16 * 12 + (uint64_t)g->n * 24;
  if (g->weighted) b += GN * kLanes * 8 + GN * 28 + GN * 5 * 8 + (uint64_t)groups * (uint64_t)g->m * 8;
  else b += GN * sizeof(MaskRec);
  return b;
}

}  // namespace bcd

extern "C" {

double bcd_server_now(void) { return steady_now(); }

bcd_status bcd_server_workspace_bytes(const bcd_graph *gh, int32_t groups, int32_t workers, uint64_t *bytes) {
  BCD_GUARD_BEGIN
  if (!gh || !bytes) return fail(BCD_ERR_INVALID_ARG, "NULL argument");
  const Graph *g = reinterpret_cast<const Graph *>(gh);
  if (groups <= 0) groups = g->config().groups;
  if (workers <= 0) workers = 2;
  *bytes = batch_workspace_bytes(g, groups) * (uint64_t)workers;
  return BCD_OK;
  BCD_GUARD_END
}

bcd_status bcd_server_create(const bcd_graph *gh, const bcd_server_config *cfg, bcd_server **out) {
  BCD_GUARD_BEGIN
  if (!gh || !out) return fail(BCD_ERR_INVALID_ARG, "NULL argument");
  Graph *g = const_cast<Graph *>(reinterpret_cast<const Graph *>(gh));
  std::unique_ptr<bcd_server> S(new (std::nothrow) bcd_server());
  if (!S) return fail(BCD_ERR_OUT_OF_MEMORY, "host allocation failed");
  S->g = g;
  if (cfg) S->cfg = *cfg;
  if (S->cfg.hbm_budget_bytes == 0) S->cfg.hbm_budget_bytes = 64ull << 30;
  if (S->cfg.workers <= 0) S->cfg.workers = 2;
  if (S->cfg.workers > 16) return fail(BCD_ERR_INVALID_ARG, "at most 16 workers");
  if (S->cfg.groups <= 0) S->cfg.groups = g->config().groups;
  if (S->cfg.queue_capacity <= 0) S->cfg.queue_capacity = 4096;
  if ((uint64_t)S->cfg.groups * (uint64_t)g->n >= (1ull << 32))
    return fail(BCD_ERR_INVALID_ARG, "groups * n must stay below 2^32");
  const uint64_t fixed = batch_workspace_bytes(g, S->cfg.groups) * (uint64_t)S->cfg.workers;
  if (fixed >= S->cfg.hbm_budget_bytes)
    return fail(BCD_ERR_OUT_OF_MEMORY, "HBM budget smaller than the batch workspaces (" + std::to_string(fixed) +
                                           " bytes); lower groups or workers");
  S->budget_q = (size_t)(S->cfg.hbm_budget_bytes - fixed);
  // the server brings its own workspaces: idle ones pooled by earlier calls
  // on this graph give their memory back first
  g->trim_pool();
  S->plan_ws.reset(new (std::nothrow) Workspace());
  if (!S->plan_ws) return fail(BCD_ERR_OUT_OF_MEMORY, "host allocation failed");
  STCHK(S->plan_ws->init_common(g));
  STCHK(S->plan_ws->ensure_reach());
  for (int i = 0; i < S->cfg.workers; ++i) {
    std::unique_ptr<Workspace> w(new (std::nothrow) Workspace());
    if (!w) return fail(BCD_ERR_OUT_OF_MEMORY, "host allocation failed");
    STCHK(w->init_common(g));
    STCHK(w->ensure_batch(S->cfg.groups));
    if (g->weighted) STCHK(w->ensure_weighted());
    S->wss.push_back(std::move(w));
  }
  bcd_server *raw = S.get();
  try {
    raw->planner = std::thread(planner_loop, raw);
    for (auto &w : raw->wss) raw->workers.emplace_back(worker_loop, raw, w.get());
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(raw->mu);
      raw->stop = true;
    }
    raw->cv_plan.notify_all();
    raw->cv_work.notify_all();
    if (raw->planner.joinable()) raw->planner.join();
    for (auto &t : raw->workers) t.join();
    return fail(BCD_ERR_OUT_OF_MEMORY, "thread start failed");
  }
  *out = S.release();
  return BCD_OK;
  BCD_GUARD_END
}

bcd_status bcd_server_submit(bcd_server *S, const bcd_query *q, uint64_t *ticket) {
  BCD_GUARD_BEGIN
  if (!S || !q || !ticket) return fail(BCD_ERR_INVALID_ARG, "NULL argument");
  Graph *g = S->g;
  if (q->kind == BCD_QUERY_EXACT || q->kind == BCD_QUERY_SAMPLED) {
    if (q->r < 0 || q->r >= g->n) return fail(BCD_ERR_INVALID_ARG, "r out of range");
    if (q->kind == BCD_QUERY_SAMPLED && q->params.T_override <= 0) {
      if (!(q->params.eps > 0.0) || !std::isfinite(q->params.eps)) return fail(BCD_ERR_INVALID_ARG, "eps must be > 0");
      if (!(q->params.delta > 0.0 && q->params.delta < 1.0))
        return fail(BCD_ERR_INVALID_ARG, "delta must be in (0,1)");
    }
  } else if (q->kind == BCD_QUERY_SET) {
    if (!q->rs || q->l <= 0 || !q->bc_out) return fail(BCD_ERR_INVALID_ARG, "set query needs rs, l > 0, bc_out");
    for (int64_t i = 0; i < q->l; ++i)
      if (q->rs[i] < 0 || q->rs[i] >= g->n) return fail(BCD_ERR_INVALID_ARG, "target out of range");
  } else {
    return fail(BCD_ERR_INVALID_ARG, "unknown query kind");
  }
  auto sq = std::make_shared<SQuery>();
  sq->q = *q;
  if (q->kind == BCD_QUERY_SET) sq->rs.assign(q->rs, q->rs + q->l);
  sq->q.rs = nullptr;
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stop || S->closing) return fail(BCD_ERR_CANCELLED, "server is shutting down");
  if (S->outstanding >= (size_t)S->cfg.queue_capacity) return fail(BCD_ERR_AGAIN, "queue full");
  sq->ticket = S->next_ticket++;
  sq->res.ticket = sq->ticket;
  sq->res.tag = q->tag;
  sq->res.kind = q->kind;
  sq->res.t_arrive_s = steady_now();
  S->outstanding++;
  S->submitted.push_back(sq);
  S->cv_plan.notify_all();
  *ticket = sq->ticket;
  return BCD_OK;
  BCD_GUARD_END
}

bcd_status bcd_server_poll(bcd_server *S, bcd_result *out, int32_t cap, int32_t *n_out, int64_t timeout_ns) {
  BCD_GUARD_BEGIN
  if (!S || !out || cap <= 0 || !n_out) return fail(BCD_ERR_INVALID_ARG, "bad argument");
  std::unique_lock<std::mutex> lk(S->mu);
  if (S->finished.empty() && timeout_ns != 0) {
    if (timeout_ns < 0) S->cv_done.wait(lk, [&] { return !S->finished.empty(); });
    else S->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), [&] { return !S->finished.empty(); });
  }
  int32_t k = 0;
  while (k < cap && !S->finished.empty()) {
    out[k++] = S->finished.front();
    S->finished.pop_front();
    S->outstanding--;
  }
  *n_out = k;
  if (k == 0) return fail(BCD_ERR_AGAIN, "no result ready");
  return BCD_OK;
  BCD_GUARD_END
}

bcd_status bcd_server_get_stats(bcd_server *S, bcd_server_stats *out) {
  BCD_GUARD_BEGIN
  if (!S || !out) return fail(BCD_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->stats;
  return BCD_OK;
  BCD_GUARD_END
}

bcd_status bcd_server_shutdown(bcd_server *S) {
  BCD_GUARD_BEGIN
  if (!S) return fail(BCD_ERR_INVALID_ARG, "NULL argument");
  std::unique_lock<std::mutex> lk(S->mu);
  S->closing = true;
  // queries not yet taken by the planner are cancelled now; the planner
  // cancels the one it holds unless it was already admitted
  for (auto &q : S->submitted) post_result(S, q, BCD_ERR_CANCELLED);
  S->submitted.clear();
  S->cv_plan.notify_all();
  // admitted queries run to completion (their batches may already be in flight)
  S->cv_drained.wait(lk, [&] { return !S->planning && S->submitted.empty() && S->active.empty(); });
  return BCD_OK;
  BCD_GUARD_END
}

bcd_status bcd_server_destroy(bcd_server *S) {
  BCD_GUARD_BEGIN
  if (!S) return BCD_OK;
  (void)bcd_server_shutdown(S);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_plan.notify_all();
  S->cv_work.notify_all();
  if (S->planner.joinable()) S->planner.join();
  for (auto &t : S->workers) t.join();
  // whatever did not finish is cancelled
  for (auto &q : S->active) {
    if (q->dres) (void)hipFree(q->dres);
    q->dres = nullptr;
  }
  S->active.clear();
  S->submitted.clear();
  for (auto &c : S->cache) (void)hipFree(c.second);
  S->cache.clear();
  S->cached = 0;
  delete S;
  return BCD_OK;
  BCD_GUARD_END
}

}  // extern "C"
