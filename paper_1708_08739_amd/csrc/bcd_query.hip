// libbcd query layer: RV(r), batches of per-source passes, and the ABI
// calls built on them (Alg.1, the set form of Section 4.2, Alg.2, and the
// verification hooks).
#include <memory>
#include <thread>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/bcd.h"
#include "bcd_host_internal.h"

namespace bcd {


static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Neumaier-compensated sum in the order given (Alg.1 sums over RV(r) in
// ascending vertex order; Alg.2 in draw order).
double compensated_sum(const double *x, size_t k, size_t stride) {
  double s = 0.0, c = 0.0;
  for (size_t i = 0; i < k; ++i) {
    const double v = x[i * stride];
    const double t = s + v;
    if (std::fabs(s) >= std::fabs(v)) c += (s - t) + v;
    else c += (v - t) + s;
    s = t;
  }
  return s + c;
}

// SplitMix64 output t for state `seed` (Steele, Lea and Flood 2014), and the
// multiply-high map to [0, k).
uint64_t splitmix_at(uint64_t seed, uint64_t t) {
  uint64_t z = seed + (t + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t index_below(uint64_t x, uint64_t k) {
  return (uint64_t)(((unsigned __int128)x * (unsigned __int128)k) >> 64);
}

// ------------------------------------------------------- reachability

// Vertices reachable from `root` over the reverse graph (reverse = true,
// Def.3: the vertices that reach root) or the graph itself.  Bit v of
// `bits` is set for every vertex met, root included; *count excludes root.
bcd_status reach_set(Graph *g, Workspace *ws, int32_t root, bool reverse, std::vector<uint32_t> &bits,
                     int64_t *count, uint8_t *d_lev) {
  STCHK(ws->ensure_reach());
  const int64_t n = g->n;
  const size_t words = (size_t)(n + 31) / 32;
  hipStream_t st = ws->stream;
  const int64_t *rp = reverse ? g->d_irp : g->d_rp;
  const int32_t *col = reverse ? g->d_icol : g->d_col;
  // the other direction, for levels found bottom-up
  const int64_t *rpo = reverse ? g->d_rp : g->d_irp;
  const int32_t *colo = reverse ? g->d_col : g->d_icol;
  Launch L = g->launch();
  if (!d_lev && lds_reach_fits(g)) {
    // small graph: the whole traversal in one workgroup, one launch
    HIPCHK(launch_lds_reach(g, rp, col, root, ws->bitmap, st));
    HIPCHK(hipMemcpyAsync(ws->h_bitmap, ws->bitmap, words * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    bits.assign(ws->h_bitmap, ws->h_bitmap + words);
    int64_t c = 0;
    for (size_t i = 0; i < words; ++i) c += __builtin_popcount(bits[i]);
    *count = c - 1;
    return BCD_OK;
  }
  HIPCHK(hipMemsetAsync(ws->bitmap, 0, words * sizeof(uint32_t), st));
  // per queue c: its length at rqn[4c], the arcs of its vertices (uint64) at rqn[4c + 2]
  HIPCHK(hipMemsetAsync(ws->rqn, 0, 8 * sizeof(uint32_t), st));
  auto qlen = [&](int c) { return ws->rqn + 4 * c; };
  auto qarcs = [&](int c) { return reinterpret_cast<uint64_t *>(ws->rqn + 4 * c + 2); };
  HIPCHK(launch_reach_init(ws->bitmap, ws->rq[0], qlen(0), root, st));
  int cur = 0;
  const int chunk = 8;
  // a level whose frontier has at least m/64 arcs to scan is found bottom-up
  // (Beamer's direction switch), unless levels are wanted: at R-MAT 22 the
  // two largest levels of RV(r) take about 60 M in-arc checks top-down and
  // far fewer out-arc checks bottom-up.  The rule counts arcs, not vertices:
  // the second level's frontier is a few ten thousand vertices of large
  // in-degree (40 M in-arcs)
  const uint64_t bu_arcs = d_lev ? ~0ull : (uint64_t)std::max<int64_t>(64, g->m / 64);
  for (int64_t level = 0; level <= n;) {
    for (int i = 0; i < chunk; ++i, ++level) {
      HIPCHK(hipMemsetAsync(qlen(1 - cur), 0, 4 * sizeof(uint32_t), st));
      HIPCHK(launch_reach_level(rp, col, ws->bitmap, ws->rq[cur], qlen(cur), qarcs(cur), ws->rq[1 - cur],
                                qlen(1 - cur), qarcs(1 - cur), d_lev, (int)level, bu_arcs, L, st));
      if (!d_lev)
        HIPCHK(launch_reach_bu(rpo, colo, rp, ws->bitmap, qarcs(cur), ws->rq[1 - cur], qlen(1 - cur),
                               qarcs(1 - cur), n, bu_arcs, L, st));
      cur = 1 - cur;
    }
    uint32_t *h = reinterpret_cast<uint32_t *>(ws->h_misc);
    HIPCHK(hipMemcpyAsync(h, qlen(cur), sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (h[0] == 0) break;
  }
  HIPCHK(hipMemcpyAsync(ws->h_bitmap, ws->bitmap, words * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  bits.assign(ws->h_bitmap, ws->h_bitmap + words);
  int64_t c = 0;
  for (size_t i = 0; i < words; ++i) c += __builtin_popcount(bits[i]);
  *count = c - 1;
  return BCD_OK;
}

void bits_to_list(const std::vector<uint32_t> &bits, int64_t n, int32_t skip, std::vector<int32_t> &out) {
  out.clear();
  for (size_t wi = 0; wi < bits.size(); ++wi) {
    uint32_t x = bits[wi];
    while (x) {
      const int b = __builtin_ctz(x);
      x &= x - 1;
      const int64_t v = (int64_t)wi * 32 + b;
      if (v < n && v != skip) out.push_back((int32_t)v);
    }
  }
}

// ------------------------------------------------------ source order
//
// The cost of a batch grows with the number of distinct BFS levels a vertex
// has across the 64 sources of a column group.  Sources whose distances to
// a few hub vertices agree tend to agree everywhere, so batches are filled
// in the order of that distance signature.  This only decides which sources
// share a batch: each source's dependency is independent of its batch, and
// every reduction still runs in the order the paper's sums are written in.

constexpr int kLandmarks = 16;

static bcd_status ensure_landmarks(Graph *g, Workspace *ws) {
  std::lock_guard<std::mutex> lk(g->lm_mu);
  if (g->lm_ready) return BCD_OK;
  const int64_t n = g->n;
  // the kLandmarks vertices of largest in-degree (ties: smaller id)
  std::vector<int64_t> indeg((size_t)n, 0);
  {
    std::vector<int64_t> irp((size_t)n + 1);
    HIPCHK(hipMemcpy(irp.data(), g->d_irp, ((size_t)n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
    for (int64_t v = 0; v < n; ++v) indeg[(size_t)v] = irp[(size_t)v + 1] - irp[(size_t)v];
  }
  std::vector<int32_t> ids((size_t)n);
  for (int64_t v = 0; v < n; ++v) ids[(size_t)v] = (int32_t)v;
  const int k = (int)std::min<int64_t>(kLandmarks, n);
  std::partial_sort(ids.begin(), ids.begin() + k, ids.end(), [&](int32_t a, int32_t b) {
    return indeg[(size_t)a] != indeg[(size_t)b] ? indeg[(size_t)a] > indeg[(size_t)b] : a < b;
  });
  g->lm_sig.assign((size_t)n * kLandmarks, 255);
  uint8_t *d_lev = nullptr;
  if (hipMalloc((void **)&d_lev, (size_t)n) != hipSuccess) {
    (void)hipGetLastError();
    return fail(BCD_ERR_OUT_OF_MEMORY, "landmark level buffer");
  }
  std::vector<uint8_t> lev((size_t)n);
  std::vector<uint32_t> bits;
  bcd_status rc = BCD_OK;
  for (int h = 0; h < k && rc == BCD_OK; ++h) {
    hipError_t e = hipMemsetAsync(d_lev, 255, (size_t)n, ws->stream);
    if (e != hipSuccess) {
      rc = hip_fail(e, "landmark reset");
      break;
    }
    int64_t cnt = 0;
    // distance from every vertex to the hub = BFS level from the hub on the reverse graph
    rc = reach_set(g, ws, ids[(size_t)h], true, bits, &cnt, d_lev);
    if (rc != BCD_OK) break;
    e = hipMemcpy(lev.data(), d_lev, (size_t)n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      rc = hip_fail(e, "landmark copy");
      break;
    }
    lev[(size_t)ids[(size_t)h]] = 0;
    for (int64_t v = 0; v < n; ++v) g->lm_sig[(size_t)v * kLandmarks + h] = lev[(size_t)v];
  }
  (void)hipFree(d_lev);
  if (rc == BCD_OK) g->lm_ready = true;
  return rc;
}

// Processing order (positions into src) for the batched engines.
bcd_status source_order(Graph *g, Workspace *ws, const std::vector<int32_t> &src, std::vector<uint32_t> &ord) {
  ord.resize(src.size());
  for (size_t i = 0; i < src.size(); ++i) ord[i] = (uint32_t)i;
  if (src.size() <= (size_t)kLanes || g->n < 4096) return BCD_OK;
  STCHK(ensure_landmarks(g, ws));
  const uint8_t *sig = g->lm_sig.data();
  const size_t ns = src.size();
  // ties keep ascending source order: start from it (the lists are usually
  // ascending already), then a stable LSD radix sort over the signature
  // bytes, last byte first, gives the lexicographic signature order
  if (!std::is_sorted(src.begin(), src.end()))
    std::stable_sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t b) { return src[a] < src[b]; });
  std::vector<uint8_t> key(ns * kLandmarks);  // by position in src, contiguous
  for (size_t i = 0; i < ns; ++i) std::memcpy(&key[i * kLandmarks], sig + (size_t)src[i] * kLandmarks, kLandmarks);
  std::vector<uint32_t> tmp(ns);
  for (int byte = kLandmarks - 1; byte >= 0; --byte) {
    size_t cnt[257] = {0};
    for (size_t i = 0; i < ns; ++i) ++cnt[(size_t)key[(size_t)ord[i] * kLandmarks + byte] + 1];
    bool constant = false;  // every key has the same byte here: the pass is the identity
    for (int d = 1; d <= 256; ++d) constant = constant || cnt[d] == ns;
    if (constant) continue;
    for (int d = 1; d <= 256; ++d) cnt[d] += cnt[d - 1];
    for (size_t i = 0; i < ns; ++i) tmp[cnt[key[(size_t)ord[i] * kLandmarks + byte]]++] = ord[i];
    ord.swap(tmp);
  }
  return BCD_OK;
}

// --------------------------------------------------------- targets


// -------------------------------------------------- batched engine

struct BatchExport {
  uint64_t *dist = nullptr;  // device [k][n]
  unsigned long long *sigma = nullptr;
  double *delta = nullptr;
  int64_t k = 0;
};

// One batch: `k` sources already staged in ws->h_items0 / h_masks0 (lane i
// of the batch is group i/64, lane i%64).  Runs the forward levels until the
// next level is empty, the backward levels down to the shallowest target level (or
// level 0 when `full`), copies the per-lane target dependencies into
// ws->h_res, and leaves the state clean for the next batch.
static bcd_status run_one_batch(Graph *g, Workspace *ws, int k, int ntgt, bool full, BatchExport *ex,
                                ProfAcc *prof, bool *sigma_overflow, bool copy_res = true,
                                unsigned long long *ovl_out = nullptr) {
  hipStream_t st = ws->stream;
  const DevGraph D = g->dev();
  const bool profiling = g->profiling.load();
  const size_t G64 = (size_t)ws->G * kLanes;
  HIPCHK(hipMemcpyAsync(ws->d_items0, ws->h_items0, (size_t)k * sizeof(uint32_t), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(ws->d_masks0, ws->h_masks0, (size_t)k * sizeof(unsigned long long), hipMemcpyHostToDevice,
                        st));
  const int push = g->config().push;
  if (push && !ws->sig_zero) {
    // counts pulled by an earlier batch on this workspace: clear them all once
    HIPCHK(hipMemsetAsync(ws->S.sig, 0, (size_t)ws->G * (size_t)ws->n * kLanes * sizeof(unsigned long long), st));
  }
  ws->sig_zero = false;  // until this batch has completed
  for (int attempt = 0;; ++attempt) {
    ws->S.epoch += 1;
    BatchState S = ws->S;  // kernel arguments: this batch's epoch and capacity
    if (!ex) S.dout = nullptr;
    S.P = ws->batch_parts(k);  // partitions that hold this batch's groups
    S.gused = (k + kLanes - 1) / kLanes;
    S.last_lanes = (k % kLanes) == 0 ? ~0ull : ((1ull << (k % kLanes)) - 1ull);
    S.bu_den = g->config().bottom_up;
    S.push = push;
    S.keep_all = full ? 1 : 0;
    const int P = S.P;
    const Launch L = g->launch_parts(P);
    // level-0 placement depends on the partition sizes (they change when the list grows)
    ws->stage_sources_dest(k);
    HIPCHK(hipMemcpyAsync(ws->d_dest0, ws->h_dest0, (size_t)k * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    uint32_t *hc = ws->h_cnt;
    uint32_t *hc0 = hc + kCntStage;
    for (int p = 0; p < P; ++p) hc0[p] = ws->h_cnt0[p];
    HIPCHK(hipMemcpyAsync(&S.cnt[0], hc0, (size_t)P * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    if (ntgt > 0) HIPCHK(hipMemsetAsync(S.res, 0, (size_t)ntgt * G64 * sizeof(double), st));
    HIPCHK(hipMemsetAsync(S.tmin, 0xFF, sizeof(uint32_t), st));
    HIPCHK(hipMemsetAsync(S.flags, 0, 4 * sizeof(uint32_t), st));
    HIPCHK(hipMemsetAsync(S.ovl, 0, (size_t)ws->G * sizeof(unsigned long long), st));
    HIPCHK(launch_batch_init(S, ws->d_items0, ws->d_masks0, ws->d_dest0, k, st));

    // forward, in chunks of levels between host checks; a level found
    // bottom-up gets its own kernel, launched before the level's top-down
    // kernel (both decide on the device whether they have work)
    std::vector<uint32_t> cntp(hc0, hc0 + P);  // cntp[l * P + p] = items of partition p on level l
    uint64_t last_tot = (uint64_t)k;           // items of the last recorded level
    int lmax = -1;
    int level = 0;
    int chunk = std::min(kLevelChunkMax, std::max(4, ws->last_depth + 2));
    uint32_t flags_h[2] = {0, 0}, tmin_h = 0xFFFFFFFFu;
    size_t ev = 0;
    while (lmax < 0) {
      int launched = 0;
      for (; launched < chunk && level <= g->n; ++launched, ++level) {
        if (S.bu_den > 0 && level >= 2) {
          if (profiling) HIPCHK(hipEventRecord(ws->event_pair(ev).first, st));
          HIPCHK(launch_bu_level(D, S, level, L, st));
          if (profiling) {
            HIPCHK(hipEventRecord(ws->event_pair(ev).second, st));
            ++ev;
          }
        }
        if (profiling) HIPCHK(hipEventRecord(ws->event_pair(ev).first, st));
        HIPCHK(launch_fwd_level(D, S, level, L, st));
        if (profiling) {
          HIPCHK(hipEventRecord(ws->event_pair(ev).second, st));
          ++ev;
        }
      }
      // counts of the levels not recorded yet, up to the one the last
      // launch discovered (or that the next chunk finds bottom-up)
      const int rec_from = (int)(cntp.size() / P);
      const int nrec = level - rec_from + 1;
      HIPCHK(hipMemcpyAsync(hc, &S.cnt[(size_t)rec_from * P], (size_t)nrec * P * sizeof(uint32_t),
                            hipMemcpyDeviceToHost, st));
      uint32_t *hm = reinterpret_cast<uint32_t *>(ws->h_misc);
      HIPCHK(hipMemcpyAsync(hm, S.flags, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(hm + 2, S.tmin, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      flags_h[0] = hm[0];
      flags_h[1] = hm[1];
      tmin_h = hm[2];
      if (flags_h[1]) break;
      for (int i = 0; i < nrec; ++i) {
        const int l = rec_from + i;
        uint64_t tot = 0;
        for (int p = 0; p < P; ++p) tot += hc[(size_t)i * P + p];
        // level `level` is only counted once its bottom-up kernel has run
        if (l == level && bottom_up_rule(S.bu_den, l, last_tot, S.gused, S.n)) break;
        if (tot == 0) {
          lmax = l;
          break;
        }
        cntp.insert(cntp.end(), hc + (size_t)i * P, hc + (size_t)(i + 1) * P);
        last_tot = tot;
      }
      if (lmax < 0 && level > g->n) return fail(BCD_ERR_DEVICE, "forward pass did not terminate");
      chunk = kLevelChunkMax;
    }
    if (flags_h[1]) {
      // item list overflow: grow and redo this batch from a clean state
      STCHK(ws->reset_batch_dense());
      STCHK(ws->grow_items());
      if (attempt > 8) return fail(BCD_ERR_OUT_OF_MEMORY, "frontier item list cannot grow further");
      continue;
    }
    ws->last_depth = lmax;
    if (flags_h[0]) *sigma_overflow = true;
    const size_t fwd_events = ev;

    // backward
    int stop = -1;
    if (full) stop = 0;
    else if (ntgt > 0 && tmin_h != 0xFFFFFFFFu) stop = (int)tmin_h;
    if (stop >= 0) {
      for (int lv = lmax; lv >= stop; --lv) {
        if (profiling) HIPCHK(hipEventRecord(ws->event_pair(ev).first, st));
        HIPCHK(launch_bwd_level(D, S, lv, ntgt, full ? 1 : 0, L, st));
        if (profiling) {
          HIPCHK(hipEventRecord(ws->event_pair(ev).second, st));
          ++ev;
        }
      }
    }
    const int levels = (int)(cntp.size() / P);
    PartTotals tot{};
    for (int l = 0; l < levels; ++l)
      for (int p = 0; p < P; ++p) tot.t[p] += cntp[(size_t)l * P + p];
    if (ex) {
      std::vector<uint64_t> pos((size_t)P);
      for (int p = 0; p < P; ++p) pos[(size_t)p] = (uint64_t)p * S.capP;
      for (int l = 0; l < levels; ++l)
        for (int p = 0; p < P; ++p) {
          const uint64_t c = cntp[(size_t)l * P + p];
          HIPCHK(launch_batch_export(S, l, pos[(size_t)p], c, ws->d_lane_slot, ex->dist, ex->sigma, ex->delta, ex->k,
                                     st));
          pos[(size_t)p] += c;
        }
    }
    if (ntgt > 0 && copy_res)
      HIPCHK(hipMemcpyAsync(ws->h_res, S.res, (size_t)ntgt * G64 * sizeof(double), hipMemcpyDeviceToHost, st));
    if (ovl_out)
      HIPCHK(hipMemcpyAsync(ovl_out, S.ovl, (size_t)ws->G * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    HIPCHK(launch_batch_cleanup(S, tot, L, st));
    HIPCHK(launch_ctr_fold(S.ctr, kCtrSlots, S.acc, st));
    HIPCHK(hipMemsetAsync(S.cnt, 0, ((size_t)lmax + 2) * P * sizeof(uint32_t), st));
    HIPCHK(hipStreamSynchronize(st));
    if (profiling && prof) {
      for (size_t i = 0; i < ev; ++i) {
        prof->add(g, i < fwd_events ? 0 : 1, ws->events[i].first, ws->events[i].second);
      }
      for (int l = 0; l < levels; ++l)
        for (int p = 0; p < P; ++p) {
          prof->items[0] += cntp[(size_t)l * P + p];
          if (stop >= 0 && l >= stop) prof->items[1] += cntp[(size_t)l * P + p];
        }
    }
    ws->sig_zero = push != 0;  // the cleanup of a pushing batch zeroed the counts it set
    return BCD_OK;
  }
}

// Counters of the batches completed since the last collection (folded on the
// device after each batch), then reset.
bcd_status collect_counters(Workspace *ws, uint64_t *ctr /*[C_COUNT]*/, uint64_t *dev_acc) {
  hipStream_t st = ws->stream;
  HIPCHK(hipMemcpyAsync(ws->h_ctr, dev_acc, (size_t)C_COUNT * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemsetAsync(dev_acc, 0, (size_t)C_COUNT * sizeof(uint64_t), st));
  HIPCHK(hipStreamSynchronize(st));
  for (int k = 0; k < C_COUNT; ++k) ctr[k] = ws->h_ctr[k];
  return BCD_OK;
}

static void add_profile(Graph *g, const ProfAcc &p, const uint64_t *ctr) {
  // Algorithmic bytes (per (source, element) pair, independent of how the
  // kernels share reads across sources):
  //   forward : 32 per (source, vertex) + 8 per (source, arc) + 8 per (source, DAG arc)
  //   backward: 32 per (source, vertex) + 8 per (source, arc) + 8 per (source, DAG arc)
  // of which the graph structure is 16 per vertex (its two row offsets) and
  // 4 per arc (its column index).  Counted once per work item (64 sources of
  // a column group at one vertex and level) instead of once per source, the
  // structure gives the schedule-aware figure.
  const double fb = 32.0 * ctr[C_FWD_VPAIRS] + 8.0 * ctr[C_FWD_APAIRS] + 8.0 * ctr[C_FWD_DPAIRS];
  const double bb = 32.0 * ctr[C_BWD_VPAIRS] + 8.0 * ctr[C_BWD_APAIRS] + 8.0 * ctr[C_BWD_DPAIRS];
  const bool per_item = ctr[C_FWD_ITEMS] > 0;  // the batched kernels count items on the device
  const double fs = per_item ? 16.0 * ctr[C_FWD_ITEMS] + 4.0 * ctr[C_FWD_IARCS] + 16.0 * ctr[C_FWD_VPAIRS] +
                                   4.0 * ctr[C_FWD_APAIRS] + 8.0 * ctr[C_FWD_DPAIRS]
                             : fb;
  const double bs = per_item ? 16.0 * ctr[C_BWD_ITEMS] + 4.0 * ctr[C_BWD_IARCS] + 16.0 * ctr[C_BWD_VPAIRS] +
                                   4.0 * ctr[C_BWD_APAIRS] + 8.0 * ctr[C_BWD_DPAIRS]
                             : bb;
  g->add_profile(0, p.launches[0], p.ms[0], ctr + C_FWD_VPAIRS, fb, per_item ? ctr[C_FWD_ITEMS] : p.items[0],
                 &p.iv[0], ctr[C_FWD_IARCS], fs);
  g->add_profile(1, p.launches[1], p.ms[1], ctr + C_BWD_VPAIRS, bb, per_item ? ctr[C_BWD_ITEMS] : p.items[1],
                 &p.iv[1], ctr[C_BWD_IARCS], bs);
}

// The batches b = first, first + stride, ... of the ordered source list on
// one workspace (the targets installed there); each source's dependencies
// go to its own position in dep, so stripes on different workspaces never
// write the same element.
static bcd_status run_batch_stripe(Graph *g, Workspace *ws, const std::vector<int32_t> &src,
                                   const std::vector<uint32_t> &ord, const std::vector<int32_t> &tgt, size_t first,
                                   size_t stride, std::vector<double> &dep, ProfAcc &prof, bool &ovf) {
  const int ntgt = (int)tgt.size();
  const size_t G64 = (size_t)ws->G * kLanes;
  const size_t ns = src.size();
  TargetMap tm;
  STCHK(tm.install(ws, tgt));
  std::vector<int32_t> bsrc(G64);
  for (size_t b0 = first * G64; b0 < ns; b0 += stride * G64) {
    const int k = (int)std::min(G64, ns - b0);
    for (int i = 0; i < k; ++i) bsrc[(size_t)i] = src[ord[b0 + i]];
    ws->stage_sources(bsrc.data(), k);
    STCHK(run_one_batch(g, ws, k, ntgt, false, nullptr, &prof, &ovf));
    for (int i = 0; i < k; ++i)
      for (int t = 0; t < ntgt; ++t) dep[(size_t)ord[b0 + i] * ntgt + t] = ws->h_res[(size_t)t * G64 + i];
  }
  return BCD_OK;
}

// A second workspace runs every other batch on its own stream from a helper
// thread, so one batch's host steps (result copy, staging, the level-count
// checks) and its small tail levels overlap the other's kernels.  It is taken
// from the graph's pool if one is there with the same width, else allocated
// only when HBM keeps kPipelineHeadroom free beside it (the pair then stays
// pooled with the graph; a server releases idle pooled workspaces).
constexpr uint64_t kPipelineHeadroom = 16ull << 30;

void ProfAcc::add(const Graph *g, int kind, hipEvent_t a, hipEvent_t b) {
  float ms = 0, t0 = 0, t1 = 0;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  this->ms[kind] += ms;
  launches[kind] += 1;
  if (g->prof_ref && hipEventElapsedTime(&t0, g->prof_ref, a) == hipSuccess &&
      hipEventElapsedTime(&t1, g->prof_ref, b) == hipSuccess)
    iv[kind].emplace_back((double)t0, (double)t1);
  else
    (void)hipGetLastError();
}

bcd_status run_pipelined(Graph *g, Workspace *ws, size_t nbatches, const std::function<bcd_status(Workspace *)> &prepare,
                         const StripeFn &stripe, ProfAcc &prof, bool &ovf, uint64_t *tot) {
  std::unique_ptr<Lease> ls2;
  Workspace *ws2 = nullptr;
  if (nbatches > 1) {
    ls2.reset(new (std::nothrow) Lease(g));
    bool room = ls2 && ls2->ok() && (*ls2)->batch_ready && (*ls2)->G == ws->G &&
                (!g->weighted || (*ls2)->weighted_ready);
    if (!room && ls2 && ls2->ok()) {
      size_t free_b = 0, total_b = 0;
      room = hipMemGetInfo(&free_b, &total_b) == hipSuccess &&
             (uint64_t)free_b >= batch_workspace_bytes(g, ws->G) + kPipelineHeadroom;
    }
    if (room && (*ls2)->init_common(g) == BCD_OK && prepare(ls2->w.get()) == BCD_OK && (*ls2)->G == ws->G)
      ws2 = ls2->w.get();
    else
      (void)hipGetLastError();  // run on one workspace
  }
  if (ws2) {
    bcd_status rc2 = BCD_OK;
    std::string err2;
    ProfAcc prof2;
    bool ovf2 = false;
    std::thread helper;
    try {
      helper = std::thread([&] {
        try {
          rc2 = stripe(ws2, 1, 2, prof2, ovf2);
          if (rc2 != BCD_OK) err2 = bcd_last_error();
        } catch (const std::bad_alloc &) {
          rc2 = BCD_ERR_OUT_OF_MEMORY;
          err2 = "host allocation failed";
        } catch (...) {
          rc2 = BCD_ERR_DEVICE;
          err2 = "unexpected host exception";
        }
      });
    } catch (...) {
      ws2 = nullptr;
    }
    if (ws2) {
      bcd_status rc1 = BCD_OK;
      try {
        rc1 = stripe(ws, 0, 2, prof, ovf);
      } catch (...) {  // the helper is joined before the exception goes on
        helper.join();
        throw;
      }
      helper.join();
      STCHK(rc1);
      if (rc2 != BCD_OK) return fail(rc2, err2);
      prof.merge(prof2);
      ovf = ovf || ovf2;
      uint64_t t2[C_COUNT] = {0};
      STCHK(collect_counters(ws2, t2, ws2->S.acc));
      for (int j = 0; j < C_COUNT; ++j) tot[j] += t2[j];
      return BCD_OK;
    }
  }
  return stripe(ws, 0, 1, prof, ovf);
}

static bcd_status run_batched(Graph *g, Workspace *ws, const std::vector<int32_t> &src,
                              const std::vector<int32_t> &tgt, bool want_counters, SourceRun &out) {
  const bcd_config cfg = g->config();
  STCHK(ws->ensure_batch(cfg.groups));
  const int ntgt = (int)tgt.size();
  const size_t G64 = (size_t)ws->G * kLanes;
  STCHK(ws->ensure_res((size_t)std::max(ntgt, 1) * G64));
  const size_t ns = src.size();
  out.dep.assign(ns * (size_t)std::max(ntgt, 0), 0.0);
  if (want_counters) out.counters.assign(ns * 3, 0);
  out.width = want_counters ? 1 : (int32_t)G64;
  ProfAcc prof;
  bool ovf = false;
  uint64_t tot[C_COUNT] = {0};
  std::vector<uint32_t> ord;
  STCHK(source_order(g, ws, src, ord));
  if (!want_counters) {
    auto prepare = [&](Workspace *w) -> bcd_status {
      STCHK(w->ensure_batch(cfg.groups));
      return w->ensure_res((size_t)std::max(ntgt, 1) * G64);
    };
    auto stripe = [&](Workspace *w, size_t first, size_t stride, ProfAcc &p, bool &o) -> bcd_status {
      return run_batch_stripe(g, w, src, ord, tgt, first, stride, out.dep, p, o);
    };
    STCHK(run_pipelined(g, ws, (ns + G64 - 1) / G64, prepare, stripe, prof, ovf, tot));
  }
  // counters per source need one source per batch
  TargetMap tm;
  if (want_counters) STCHK(tm.install(ws, tgt));
  for (size_t b0 = 0; want_counters && b0 < ns; b0 += 1) {
    const size_t per = 1;
    const int k = (int)std::min(per, ns - b0);
    std::vector<int32_t> bsrc((size_t)k);
    for (int i = 0; i < k; ++i) bsrc[(size_t)i] = src[ord[b0 + i]];
    ws->stage_sources(bsrc.data(), k);
    STCHK(run_one_batch(g, ws, k, ntgt, false, nullptr, &prof, &ovf));
    for (int i = 0; i < k; ++i)
      for (int t = 0; t < ntgt; ++t) out.dep[(size_t)ord[b0 + i] * ntgt + t] = ws->h_res[(size_t)t * G64 + i];
    if (want_counters) {
      uint64_t c[C_COUNT];
      STCHK(collect_counters(ws, c, ws->S.acc));
      out.counters[(size_t)ord[b0] * 3 + 0] = c[C_FWD_VPAIRS];
      out.counters[(size_t)ord[b0] * 3 + 1] = c[C_FWD_APAIRS];
      out.counters[(size_t)ord[b0] * 3 + 2] = c[C_FWD_DPAIRS];
      for (int j = 0; j < C_COUNT; ++j) tot[j] += c[j];
    }
  }
  if (!want_counters) {
    uint64_t t1[C_COUNT] = {0};
    STCHK(collect_counters(ws, t1, ws->S.acc));
    for (int j = 0; j < C_COUNT; ++j) tot[j] += t1[j];
  }
  out.te = tot[C_FWD_APAIRS];
  out.reached = tot[C_FWD_VPAIRS];
  out.dag = tot[C_FWD_DPAIRS];
  if (g->profiling.load()) add_profile(g, prof, tot);
  if (ovf) return fail(BCD_ERR_SIGMA_OVERFLOW, "a shortest-path count exceeded 2^64 - 1");
  return BCD_OK;
}

// ---------------------------------------------------- plain engine

// One source through the plain kernels.  Targets' dependencies go to
// dep[0..ntgt-1]; with `full`, the backward runs to level 0 and the whole
// state can be exported before cleanup.
static bcd_status run_plain_one(Graph *g, Workspace *ws, int32_t s, const int32_t *d_tgt, int ntgt,
                                const std::vector<int32_t> &tgt, bool full, double *dep, uint64_t *dist,
                                unsigned long long *sigma, double *delta, ProfAcc *prof, bool *ovf) {
  PlainState &P = ws->P;
  hipStream_t st = ws->stream;
  const DevGraph D = g->dev();
  const Launch L = g->launch();
  const bool profiling = g->profiling.load();
  HIPCHK(hipMemsetAsync(P.flags, 0, 4 * sizeof(uint32_t), st));
  HIPCHK(launch_plain_init(P, s, st));
  std::vector<uint32_t> cnt{1u};
  int lmax = -1, level = 0;
  int chunk = std::min(kLevelChunkMax, std::max(4, ws->last_depth + 2));
  size_t ev = 0;
  uint32_t *hc = ws->h_cnt;
  while (lmax < 0) {
    const int first = level;
    int launched = 0;
    for (; launched < chunk && level <= g->n; ++launched, ++level) {
      if (profiling) HIPCHK(hipEventRecord(ws->event_pair(ev).first, st));
      HIPCHK(launch_plain_fwd(D, P, level, L, st));
      if (profiling) {
        HIPCHK(hipEventRecord(ws->event_pair(ev).second, st));
        ++ev;
      }
    }
    HIPCHK(hipMemcpyAsync(hc, &P.cnt[first + 1], (size_t)launched * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < launched; ++i) {
      if (hc[i] == 0) {
        lmax = first + i;
        break;
      }
      cnt.push_back(hc[i]);
    }
    if (lmax < 0 && level > g->n) return fail(BCD_ERR_DEVICE, "forward pass did not terminate");
    chunk = kLevelChunkMax;
  }
  ws->last_depth = lmax;
  const size_t fwd_events = ev;
  // distances of the targets decide where the backward may stop
  int stop = full ? 0 : -1;
  std::vector<int32_t> tdist(ntgt, -1);
  if (!full && ntgt > 0) {
    std::vector<int32_t> h(ntgt);
    // gather distances through the export path of the plain state
    int32_t *dbuf = nullptr;
    if (hipMalloc((void **)&dbuf, (size_t)ntgt * sizeof(int32_t)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(BCD_ERR_OUT_OF_MEMORY, "target distance buffer");
    }
    hipError_t e = launch_plain_gather(P, d_tgt, ntgt, dbuf, nullptr, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), dbuf, (size_t)ntgt * sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(dbuf);
    if (e != hipSuccess) return hip_fail(e, "target distances");
    for (int t = 0; t < ntgt; ++t) {
      tdist[t] = h[t];
      if (h[t] > 0 && (stop < 0 || h[t] < stop)) stop = h[t];
    }
  }
  if (stop >= 0) {
    for (int lv = lmax; lv >= stop; --lv) {
      if (profiling) HIPCHK(hipEventRecord(ws->event_pair(ev).first, st));
      HIPCHK(launch_plain_bwd(D, P, lv, -1, 0, L, st));
      if (profiling) {
        HIPCHK(hipEventRecord(ws->event_pair(ev).second, st));
        ++ev;
      }
    }
  }
  if (ntgt > 0 && dep) {
    double *dbuf = nullptr;
    if (hipMalloc((void **)&dbuf, (size_t)ntgt * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(BCD_ERR_OUT_OF_MEMORY, "target dependency buffer");
    }
    std::vector<double> h(ntgt);
    hipError_t e = launch_plain_gather(P, d_tgt, ntgt, nullptr, dbuf, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), dbuf, (size_t)ntgt * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(dbuf);
    if (e != hipSuccess) return hip_fail(e, "target dependencies");
    for (int t = 0; t < ntgt; ++t)
      dep[t] = (tgt[t] == s || stop < 0 || (!full && tdist[t] <= 0)) ? 0.0 : h[t];
  }
  if (dist || sigma || delta) HIPCHK(launch_plain_export(P, 0, dist, sigma, delta, st));
  uint64_t total = 0;
  for (uint32_t c : cnt) total += c;
  HIPCHK(launch_plain_cleanup(P, total, st));
  HIPCHK(launch_ctr_fold(P.ctr, kCtrSlots, P.acc, st));
  HIPCHK(hipMemsetAsync(P.cnt, 0, ((size_t)lmax + 2) * sizeof(uint32_t), st));
  HIPCHK(hipMemcpyAsync(ws->h_misc, P.flags, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (reinterpret_cast<uint32_t *>(ws->h_misc)[0]) *ovf = true;
  if (profiling && prof) {
    for (size_t i = 0; i < ev; ++i) {
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, ws->events[i].first, ws->events[i].second));
      const int kind = i < fwd_events ? 0 : 1;
      prof->ms[kind] += ms;
      prof->launches[kind] += 1;
    }
  }
  return BCD_OK;
}

static bcd_status run_plain(Graph *g, Workspace *ws, const std::vector<int32_t> &src,
                            const std::vector<int32_t> &tgt, bool want_counters, SourceRun &out) {
  STCHK(ws->ensure_plain());
  const int ntgt = (int)tgt.size();
  int32_t *d_tgt = nullptr;
  if (ntgt > 0) {
    if (hipMalloc((void **)&d_tgt, (size_t)ntgt * sizeof(int32_t)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(BCD_ERR_OUT_OF_MEMORY, "target list");
    }
    hipError_t e = hipMemcpy(d_tgt, tgt.data(), (size_t)ntgt * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(d_tgt);
      return hip_fail(e, "target upload");
    }
  }
  const size_t ns = src.size();
  out.dep.assign(ns * (size_t)ntgt, 0.0);
  if (want_counters) out.counters.assign(ns * 3, 0);
  out.width = 1;
  ProfAcc prof;
  bool ovf = false;
  uint64_t tot[C_COUNT] = {0};
  bcd_status rc = BCD_OK;
  for (size_t i = 0; i < ns && rc == BCD_OK; ++i) {
    rc = run_plain_one(g, ws, src[i], d_tgt, ntgt, tgt, false, out.dep.data() + i * ntgt, nullptr, nullptr, nullptr,
                       &prof, &ovf);
    if (rc == BCD_OK && want_counters) {
      uint64_t c[C_COUNT];
      rc = collect_counters(ws, c, ws->P.acc);
      out.counters[i * 3 + 0] = c[C_FWD_VPAIRS];
      out.counters[i * 3 + 1] = c[C_FWD_APAIRS];
      out.counters[i * 3 + 2] = c[C_FWD_DPAIRS];
      for (int j = 0; j < C_COUNT; ++j) tot[j] += c[j];
    }
  }
  if (d_tgt) (void)hipFree(d_tgt);
  if (rc != BCD_OK) return rc;
  if (!want_counters) STCHK(collect_counters(ws, tot, ws->P.acc));
  out.te = tot[C_FWD_APAIRS];
  out.reached = tot[C_FWD_VPAIRS];
  out.dag = tot[C_FWD_DPAIRS];
  if (g->profiling.load()) add_profile(g, prof, tot);
  if (ovf) return fail(BCD_ERR_SIGMA_OVERFLOW, "a shortest-path count exceeded 2^64 - 1");
  return BCD_OK;
}

bcd_status run_staged_batch(Graph *g, Workspace *ws, int k, int ntgt, unsigned long long *ovl_out, bool *ovf,
                            ProfAcc *prof) {
  if (g->weighted) return run_staged_wbatch(g, ws, k, ntgt, ovl_out, ovf, prof);
  return run_one_batch(g, ws, k, ntgt, false, nullptr, prof, ovf, false, ovl_out);
}

void record_profile(Graph *g, const ProfAcc &p, const uint64_t *ctr) {
  if (g->weighted) record_wprofile(g, p, ctr);
  else add_profile(g, p, ctr);
}

bcd_status run_sources(Graph *g, Workspace *ws, const std::vector<int32_t> &src, const std::vector<int32_t> &tgt,
                       bool want_counters, SourceRun &out) {
  if (g->config().engine == BCD_ENGINE_LDS) return run_lds(g, ws, src, tgt, want_counters, out);
  if (g->weighted) return run_weighted(g, ws, src, tgt, want_counters, out);
  if (g->config().engine == BCD_ENGINE_PLAIN) return run_plain(g, ws, src, tgt, want_counters, out);
  return run_batched(g, ws, src, tgt, want_counters, out);
}

// ------------------------------------------------------- compression
//
// Gates (the fold that compression uses).  Call a vertex x gated into a
// when x lies on no directed cycle (its strongly connected component is
// {x}) and every out-neighbour y of x funnels into a: y = a, or y is itself
// gated into a.  Then every path from x that leaves the set H of vertices
// gated into a passes through a, and a reaches no vertex of H (a vertex of
// H reached from a would share a cycle with a).  So for a source s gated
// into a and any t outside H with t != a, every shortest s-u path to a
// vertex u beyond a is a shortest s-a path followed by a shortest a-u path:
// sigma_su = sigma_sa sigma_au and sigma_su(t) = sigma_sa sigma_au(t), and
// vertices of H contribute nothing through t.  Hence
//   delta_s(t) = delta_a(t)          (t not in H, t != a),
//   delta_s(a) = |vertices a reaches|  (every path past a passes a),
// for positive arc lengths as for unit ones.  A source with no in-arcs and
// one out-arc (s, v) is the simplest case (a = v, or v's own gate).  The
// gate is a vertex separator of s's paths valid for shortest paths in a
// digraph, in the spirit of the shattering at cut vertices the paper
// says composes with RV(r) (Section 4.2).
//
// Computed once per graph on the host: Tarjan's strongly connected
// components, iteratively, over the out-CSR; a component is completed only
// after every component it reaches, so each singleton's gate is decided
// from final gates of its out-neighbours.
static bcd_status ensure_gates(Graph *g) {
  std::lock_guard<std::mutex> lk(g->gate_mu);
  if (g->gates_ready) return BCD_OK;
  const int64_t n = g->n, m = g->m;
  std::vector<int32_t> col((size_t)std::max<int64_t>(m, 1));
  if (m > 0) HIPCHK(hipMemcpy(col.data(), g->d_col, (size_t)m * sizeof(int32_t), hipMemcpyDeviceToHost));
  const std::vector<int64_t> &rp = g->h_rp;
  std::vector<int32_t> gate((size_t)n, -1);
  std::vector<int64_t> index((size_t)n, -1), low((size_t)n, 0), edge((size_t)n, 0);
  std::vector<int32_t> stack, call;
  std::vector<uint8_t> on_stack((size_t)n, 0);
  int64_t next_index = 0;
  auto funnel = [&](int32_t y) { return gate[(size_t)y] >= 0 ? gate[(size_t)y] : y; };
  for (int64_t root = 0; root < n; ++root) {
    if (index[(size_t)root] >= 0) continue;
    call.push_back((int32_t)root);
    index[(size_t)root] = low[(size_t)root] = next_index++;
    edge[(size_t)root] = rp[(size_t)root];
    stack.push_back((int32_t)root);
    on_stack[(size_t)root] = 1;
    while (!call.empty()) {
      const int32_t v = call.back();
      if (edge[(size_t)v] < rp[(size_t)v + 1]) {
        const int32_t w = col[(size_t)edge[(size_t)v]++];
        if (index[(size_t)w] < 0) {
          index[(size_t)w] = low[(size_t)w] = next_index++;
          edge[(size_t)w] = rp[(size_t)w];
          stack.push_back(w);
          on_stack[(size_t)w] = 1;
          call.push_back(w);
        } else if (on_stack[(size_t)w]) {
          low[(size_t)v] = std::min(low[(size_t)v], index[(size_t)w]);
        }
        continue;
      }
      call.pop_back();
      if (!call.empty()) low[(size_t)call.back()] = std::min(low[(size_t)call.back()], low[(size_t)v]);
      if (low[(size_t)v] != index[(size_t)v]) continue;
      // v roots a component: pop it
      int32_t x;
      int64_t size = 0;
      do {
        x = stack.back();
        stack.pop_back();
        on_stack[(size_t)x] = 0;
        ++size;
      } while (x != v);
      if (size != 1 || rp[(size_t)v + 1] == rp[(size_t)v]) continue;
      // a singleton with out-arcs: gated if every out-neighbour funnels alike
      const int32_t a = funnel(col[(size_t)rp[(size_t)v]]);
      bool same = true;
      for (int64_t e = rp[(size_t)v] + 1; e < rp[(size_t)v + 1] && same; ++e) same = funnel(col[(size_t)e]) == a;
      if (same) gate[(size_t)v] = a;
    }
  }
  g->gate.swap(gate);
  g->gates_ready = true;
  return BCD_OK;
}

// Exact and set calls with compression on: a source s gated into a runs no
// pass when no target is gated into a (so no target lies in the set H of
// vertices gated into a): delta_s(t) = delta_a(t) for a target t != a,
// where a runs when it is a source, and otherwise reaches no target but
// itself, so delta_s(t) = 0; and delta_s(a) = the number of vertices a
// reaches.  `src` and the sources that run are ascending; dep is filled for
// all of `src`.
static bcd_status run_sources_folded(Graph *g, Workspace *ws, const std::vector<int32_t> &src,
                                     const std::vector<int32_t> &tgt, SourceRun &out, int64_t *ran) {
  if (g->config().compress == 0) {
    *ran = (int64_t)src.size();
    return run_sources(g, ws, src, tgt, false, out);
  }
  STCHK(ensure_gates(g));
  const size_t ns = src.size(), nt = tgt.size();
  // gates that some target is gated into: sources gated there run
  std::vector<int32_t> held;
  for (int32_t t : tgt)
    if (g->gate[(size_t)t] >= 0) held.push_back(g->gate[(size_t)t]);
  std::sort(held.begin(), held.end());
  auto fold_of = [&](int32_t s) {
    const int32_t a = g->gate[(size_t)s];
    return (a >= 0 && !std::binary_search(held.begin(), held.end(), a)) ? a : -1;
  };
  std::vector<int32_t> runs;
  runs.reserve(ns);
  for (int32_t s : src)
    if (fold_of(s) < 0) runs.push_back(s);
  SourceRun run;
  if (!runs.empty()) STCHK(run_sources(g, ws, runs, tgt, false, run));
  std::vector<int64_t> reach(nt, -1);  // vertices a target reaches, when needed
  out.dep.assign(ns * nt, 0.0);
  size_t j = 0;
  for (size_t i = 0; i < ns; ++i) {
    const int32_t s = src[i];
    const int32_t v = fold_of(s);
    if (v < 0) {
      for (size_t t = 0; t < nt; ++t) out.dep[i * nt + t] = run.dep[j * nt + t];
      ++j;
      continue;
    }
    const auto it = std::lower_bound(runs.begin(), runs.end(), v);
    const bool has_v = it != runs.end() && *it == v;
    const size_t jv = (size_t)(it - runs.begin());
    for (size_t t = 0; t < nt; ++t) {
      if (tgt[t] == v) {
        if (reach[t] < 0) {
          std::vector<uint32_t> bits;
          STCHK(reach_set(g, ws, v, false, bits, &reach[t], nullptr));
        }
        out.dep[i * nt + t] = (double)reach[t];
      } else {
        out.dep[i * nt + t] = has_v ? run.dep[jv * nt + t] : 0.0;
      }
    }
  }
  out.te = run.te;
  out.reached = run.reached;
  out.dag = run.dag;
  out.width = run.width;
  *ran = (int64_t)runs.size();
  return BCD_OK;
}

}  // namespace bcd

using namespace bcd;

// ------------------------------------------------------------------ ABI

static bcd_status lease_ws(Graph *g, Lease &ls) {
  if (!ls.ok()) return fail(BCD_ERR_OUT_OF_MEMORY, "workspace allocation failed");
  return ls->init_common(g);
}

extern "C" {

bcd_status bcd_rv(const bcd_graph *gh, bcd_vid r, bcd_vid *out, int64_t cap, int64_t *count) {
  BCD_GUARD_BEGIN
  if (!gh || !count) return fail(BCD_ERR_INVALID_ARG, "NULL argument");
  Graph *g = const_cast<Graph *>(reinterpret_cast<const Graph *>(gh));
  if (r < 0 || r >= g->n) return fail(BCD_ERR_INVALID_ARG, "r out of range");
  if (out && cap < 0) return fail(BCD_ERR_INVALID_ARG, "cap < 0");
  Lease ls(g);
  STCHK(lease_ws(g, ls));
  std::vector<uint32_t> bits;
  int64_t k = 0;
  STCHK(reach_set(g, ls.w.get(), r, true, bits, &k, nullptr));
  if (out && k > cap) {
    *count = k;
    return fail(BCD_ERR_BUFFER_TOO_SMALL, "RV(r) has " + std::to_string(k) + " vertices");
  }
  if (out) {
    std::vector<int32_t> list;
    bits_to_list(bits, g->n, r, list);
    std::copy(list.begin(), list.end(), out);
  }
  *count = k;
  return BCD_OK;
  BCD_GUARD_END
}

bcd_status bcd_bc_exact(const bcd_graph *gh, bcd_vid r, double *bc, bcd_stats *st) {
  BCD_GUARD_BEGIN
  if (!gh || !bc) return fail(BCD_ERR_INVALID_ARG, "NULL argument");
  Graph *g = const_cast<Graph *>(reinterpret_cast<const Graph *>(gh));
  if (r < 0 || r >= g->n) return fail(BCD_ERR_INVALID_ARG, "r out of range");
  bcd_stats s{};
  s.fr_size = -1;
  if (g->outdeg(r) == 0) {  // Prop.1
    s.rv_size = -1;
    *bc = 0.0;
    if (st) *st = s;
    return BCD_OK;
  }
  Lease ls(g);
  STCHK(lease_ws(g, ls));
  const double t0 = now_s();
  std::vector<uint32_t> bits;
  int64_t k = 0;
  STCHK(reach_set(g, ls.w.get(), r, true, bits, &k, nullptr));
  std::vector<int32_t> rv;
  bits_to_list(bits, g->n, r, rv);
  const double t1 = now_s();
  SourceRun run;
  int64_t ran = 0;
  STCHK(run_sources_folded(g, ls.w.get(), rv, std::vector<int32_t>{r}, run, &ran));
  const double v = compensated_sum(run.dep.data(), rv.size(), 1);
  const double t2 = now_s();
  s.rv_size = k;
  s.distinct_sources = ran;
  s.traversed_edges = run.te;
  s.reached = run.reached;
  s.dag_arcs = run.dag;
  s.t_rv_s = t1 - t0;
  s.t_bc_s = t2 - t1;
  s.batch_width = run.width;
  *bc = v;
  if (st) *st = s;
  return BCD_OK;
  BCD_GUARD_END
}

bcd_status bcd_bc_set(const bcd_graph *gh, const bcd_vid *rs, int64_t l, double *bc, bcd_stats *st) {
  BCD_GUARD_BEGIN
  if (!gh || !rs || !bc || l <= 0) return fail(BCD_ERR_INVALID_ARG, "bad argument");
  Graph *g = const_cast<Graph *>(reinterpret_cast<const Graph *>(gh));
  for (int64_t i = 0; i < l; ++i)
    if (rs[i] < 0 || rs[i] >= g->n) return fail(BCD_ERR_INVALID_ARG, "target out of range");
  Lease ls(g);
  STCHK(lease_ws(g, ls));
  const double t0 = now_s();
  // distinct targets, then D = union of RV(r_i) over targets with out-degree > 0
  std::vector<int32_t> tg(rs, rs + l);
  std::sort(tg.begin(), tg.end());
  tg.erase(std::unique(tg.begin(), tg.end()), tg.end());
  std::vector<uint32_t> uni((size_t)(g->n + 31) / 32, 0u), bits;
  for (int32_t r : tg) {
    if (g->outdeg(r) == 0) continue;
    int64_t k = 0;
    STCHK(reach_set(g, ls.w.get(), r, true, bits, &k, nullptr));
    bits[(size_t)r >> 5] &= ~(1u << (r & 31));
    for (size_t i = 0; i < uni.size(); ++i) uni[i] |= bits[i];
  }
  std::vector<int32_t> D;
  bits_to_list(uni, g->n, -1, D);
  const double t1 = now_s();
  SourceRun run;
  int64_t ran = 0;
  STCHK(run_sources_folded(g, ls.w.get(), D, tg, run, &ran));
  std::vector<double> per(tg.size());
  for (size_t t = 0; t < tg.size(); ++t)
    per[t] = g->outdeg(tg[t]) == 0 ? 0.0 : compensated_sum(run.dep.data() + t, D.size(), tg.size());
  for (int64_t i = 0; i < l; ++i) {
    const size_t t = (size_t)(std::lower_bound(tg.begin(), tg.end(), rs[i]) - tg.begin());
    bc[i] = per[t];
  }
  if (st) {
    bcd_stats s{};
    s.rv_size = (int64_t)D.size();
    s.fr_size = -1;
    s.distinct_sources = ran;
    s.traversed_edges = run.te;
    s.reached = run.reached;
    s.dag_arcs = run.dag;
    s.t_rv_s = t1 - t0;
    s.t_bc_s = now_s() - t1;
    s.batch_width = run.width;
    *st = s;
  }
  return BCD_OK;
  BCD_GUARD_END
}

bcd_status bcd_bc_sampled(const bcd_graph *gh, bcd_vid r, const bcd_sample_params *p, double *bc, bcd_stats *st) {
  BCD_GUARD_BEGIN
  if (!gh || !p || !bc) return fail(BCD_ERR_INVALID_ARG, "NULL argument");
  Graph *g = const_cast<Graph *>(reinterpret_cast<const Graph *>(gh));
  if (r < 0 || r >= g->n) return fail(BCD_ERR_INVALID_ARG, "r out of range");
  if (p->T_override <= 0) {
    if (!(p->eps > 0.0) || !std::isfinite(p->eps)) return fail(BCD_ERR_INVALID_ARG, "eps must be > 0");
    if (!(p->delta > 0.0 && p->delta < 1.0)) return fail(BCD_ERR_INVALID_ARG, "delta must be in (0,1)");
  }
  bcd_stats s{};
  s.fr_size = -1;
  const bool all_v = (p->flags & BCD_SAMPLE_ALL_VERTICES) != 0;
  if (g->outdeg(r) == 0) {  // Prop.1
    s.rv_size = -1;
    *bc = 0.0;
    if (st) *st = s;
    return BCD_OK;
  }
  Lease ls(g);
  STCHK(lease_ws(g, ls));
  const double t0 = now_s();
  std::vector<int32_t> rv;
  int64_t k = 0;
  if (all_v) {
    // the unpruned baseline: every vertex but r is a candidate source
    rv.reserve((size_t)g->n - 1);
    for (int64_t v = 0; v < g->n; ++v)
      if (v != r) rv.push_back((int32_t)v);
    k = (int64_t)rv.size();
  } else {
    std::vector<uint32_t> bits;
    STCHK(reach_set(g, ls.w.get(), r, true, bits, &k, nullptr));
    bits_to_list(bits, g->n, r, rv);
  }
  s.rv_size = k;
  int64_t T = p->T_override;
  if (T <= 0) {
    double K = (double)(g->n - 2);
    if (!(p->flags & BCD_K_TRIVIAL)) {
      int64_t fr = 0;
      std::vector<uint32_t> fb;
      STCHK(reach_set(g, ls.w.get(), r, false, fb, &fr, nullptr));
      s.fr_size = fr;
      K = (double)fr;
    }
    const double eps_abs = (p->flags & BCD_EPS_ABSOLUTE) ? p->eps : p->eps * (double)g->n * (double)(g->n - 1);
    STCHK(bcd_sample_count(eps_abs, p->delta, K, k, &T));
  }
  s.samples = T;
  const double t1 = now_s();
  if (k == 0) {
    *bc = 0.0;
    s.t_rv_s = t1 - t0;
    if (st) *st = s;
    return BCD_OK;
  }
  if (T >= k && !(p->flags & (BCD_NO_EXACT_FALLBACK | BCD_SAMPLE_ALL_VERTICES))) {
    SourceRun run;
    STCHK(run_sources(g, ls.w.get(), rv, std::vector<int32_t>{r}, false, run));
    *bc = compensated_sum(run.dep.data(), rv.size(), 1);
    s.ran_exact = 1;
    s.distinct_sources = (int64_t)rv.size();
    s.traversed_edges = run.te;
    s.reached = run.reached;
    s.dag_arcs = run.dag;
    s.batch_width = run.width;
  } else {
    if (T > (int64_t)1 << 40) return fail(BCD_ERR_UNSUPPORTED, "sample count too large to draw");
    // draws in order; each distinct source computed once
    std::vector<int64_t> slot((size_t)k, -1);
    std::vector<int32_t> uniq;
    std::vector<int64_t> draw((size_t)T);
    for (int64_t t = 0; t < T; ++t) {
      const uint64_t idx = index_below(splitmix_at(p->seed, (uint64_t)t), (uint64_t)k);
      if (slot[idx] < 0) {
        slot[idx] = (int64_t)uniq.size();
        uniq.push_back(rv[idx]);
      }
      draw[(size_t)t] = slot[idx];
    }
    SourceRun run;
    STCHK(run_sources(g, ls.w.get(), uniq, std::vector<int32_t>{r}, false, run));
    std::vector<double> seq((size_t)T);
    for (int64_t t = 0; t < T; ++t) seq[(size_t)t] = run.dep[(size_t)draw[(size_t)t]];
    *bc = compensated_sum(seq.data(), (size_t)T, 1) * (double)k / (double)T;
    s.distinct_sources = (int64_t)uniq.size();
    s.traversed_edges = run.te;
    s.reached = run.reached;
    s.dag_arcs = run.dag;
    s.batch_width = run.width;
  }
  s.t_rv_s = t1 - t0;
  s.t_bc_s = now_s() - t1;
  if (st) *st = s;
  return BCD_OK;
  BCD_GUARD_END
}

bcd_status bcd_bc_bcd(const bcd_graph *gh, bcd_vid r, int64_t tau, uint64_t seed, double *bc, bcd_stats *st) {
  BCD_GUARD_BEGIN
  if (tau < 1) return fail(BCD_ERR_INVALID_ARG, "tau must be >= 1");
  // T = tau draws, and the exact sum whenever |RV(r)| <= tau (T >= |RV| fallback)
  bcd_sample_params p{};
  p.seed = seed;
  p.T_override = tau;
  return bcd_bc_sampled(gh, r, &p, bc, st);
  BCD_GUARD_END
}

bcd_status bcd_dependencies(const bcd_graph *gh, bcd_vid r, const bcd_vid *sources, int64_t k, double *dep,
                            uint64_t *counters) {
  BCD_GUARD_BEGIN
  if (!gh || (k > 0 && (!sources || !dep)) || k < 0) return fail(BCD_ERR_INVALID_ARG, "bad argument");
  Graph *g = const_cast<Graph *>(reinterpret_cast<const Graph *>(gh));
  if (r < 0 || r >= g->n) return fail(BCD_ERR_INVALID_ARG, "r out of range");
  for (int64_t i = 0; i < k; ++i)
    if (sources[i] < 0 || sources[i] >= g->n) return fail(BCD_ERR_INVALID_ARG, "source out of range");
  if (k == 0) return BCD_OK;
  // distinct sources, mapped back to positions
  std::vector<int32_t> uniq(sources, sources + k);
  std::sort(uniq.begin(), uniq.end());
  uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
  Lease ls(g);
  STCHK(lease_ws(g, ls));
  SourceRun run;
  STCHK(run_sources(g, ls.w.get(), uniq, std::vector<int32_t>{r}, counters != nullptr, run));
  for (int64_t i = 0; i < k; ++i) {
    const size_t u = (size_t)(std::lower_bound(uniq.begin(), uniq.end(), sources[i]) - uniq.begin());
    dep[i] = uniq[u] == r ? 0.0 : run.dep[u];
    if (counters)
      for (int j = 0; j < 3; ++j) counters[i * 3 + j] = run.counters[u * 3 + j];
  }
  return BCD_OK;
  BCD_GUARD_END
}

bcd_status bcd_multi_source_pass(const bcd_graph *gh, const bcd_vid *sources, int64_t k, uint64_t *dist,
                                 uint64_t *sigma, double *delta) {
  BCD_GUARD_BEGIN
  if (!gh || !sources || k <= 0) return fail(BCD_ERR_INVALID_ARG, "bad argument");
  Graph *g = const_cast<Graph *>(reinterpret_cast<const Graph *>(gh));
  if (g->config().engine == BCD_ENGINE_LDS) {
    for (int64_t i = 0; i < k; ++i)
      if (sources[i] < 0 || sources[i] >= g->n) return fail(BCD_ERR_INVALID_ARG, "source out of range");
    Lease ls(g);
    STCHK(lease_ws(g, ls));
    return multi_source_pass_lds(g, ls.w.get(), sources, k, dist, sigma, delta);
  }
  if (g->weighted) return multi_source_pass_weighted(g, sources, k, dist, sigma, delta);
  const bcd_config cfg = g->config();
  if (k > (int64_t)cfg.groups * kLanes) return fail(BCD_ERR_INVALID_ARG, "k exceeds the batch width");
  for (int64_t i = 0; i < k; ++i) {
    if (sources[i] < 0 || sources[i] >= g->n) return fail(BCD_ERR_INVALID_ARG, "source out of range");
    for (int64_t j = 0; j < i; ++j)
      if (sources[j] == sources[i] && i / kLanes == j / kLanes) return fail(BCD_ERR_INVALID_ARG, "repeated source");
  }
  Lease ls(g);
  STCHK(lease_ws(g, ls));
  Workspace *ws = ls.w.get();
  STCHK(ws->ensure_batch(cfg.groups));
  STCHK(ws->ensure_dout());
  const size_t G64 = (size_t)ws->G * kLanes;
  const size_t kn = (size_t)k * (size_t)g->n;
  BatchExport ex;
  ex.k = k;
  uint64_t *dd = nullptr;
  unsigned long long *ds = nullptr;
  double *dl = nullptr;
  auto cleanup = [&]() {
    if (dd) (void)hipFree(dd);
    if (ds) (void)hipFree(ds);
    if (dl) (void)hipFree(dl);
  };
  if (hipMalloc((void **)&dd, kn * 8) != hipSuccess || hipMalloc((void **)&ds, kn * 8) != hipSuccess ||
      hipMalloc((void **)&dl, kn * 8) != hipSuccess) {
    (void)hipGetLastError();
    cleanup();
    return fail(BCD_ERR_OUT_OF_MEMORY, "export buffers");
  }
  hipStream_t st = ws->stream;
  std::vector<int32_t> slot(G64, -1);
  for (int64_t i = 0; i < k; ++i) slot[(size_t)i] = (int32_t)i;
  hipError_t e = hipMemcpyAsync(ws->d_lane_slot, slot.data(), G64 * sizeof(int32_t), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(dd, 0xFF, kn * 8, st);
  if (e == hipSuccess) e = hipMemsetAsync(ds, 0, kn * 8, st);
  if (e == hipSuccess) e = hipMemsetAsync(dl, 0, kn * 8, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "export setup");
  }
  ws->stage_sources(sources, (int)k);
  ex.dist = dd;
  ex.sigma = ds;
  ex.delta = dl;
  bool ovf = false;
  ProfAcc prof;
  bcd_status rc = run_one_batch(g, ws, (int)k, 0, true, &ex, &prof, &ovf);
  if (rc == BCD_OK) {
    e = hipSuccess;
    if (dist) e = hipMemcpy(dist, dd, kn * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess && sigma) e = hipMemcpy(sigma, ds, kn * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess && delta) e = hipMemcpy(delta, dl, kn * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = hip_fail(e, "export copy");
  }
  cleanup();
  uint64_t c[C_COUNT];
  if (rc == BCD_OK) rc = collect_counters(ws, c, ws->S.acc);
  if (rc == BCD_OK && ovf) rc = fail(BCD_ERR_SIGMA_OVERFLOW, "a shortest-path count exceeded 2^64 - 1");
  return rc;
  BCD_GUARD_END
}

bcd_status bcd_source_pass(const bcd_graph *gh, bcd_vid s, uint64_t *dist, uint64_t *sigma, double *delta) {
  BCD_GUARD_BEGIN
  if (!gh) return fail(BCD_ERR_INVALID_ARG, "graph is NULL");
  Graph *g = const_cast<Graph *>(reinterpret_cast<const Graph *>(gh));
  if (s < 0 || s >= g->n) return fail(BCD_ERR_INVALID_ARG, "s out of range");
  if (g->weighted || g->config().engine != BCD_ENGINE_PLAIN) return bcd_multi_source_pass(gh, &s, 1, dist, sigma, delta);
  Lease ls(g);
  STCHK(lease_ws(g, ls));
  Workspace *ws = ls.w.get();
  STCHK(ws->ensure_plain());
  const size_t n = (size_t)g->n;
  uint64_t *dd = nullptr;
  unsigned long long *ds = nullptr;
  double *dl = nullptr;
  auto cleanup = [&]() {
    if (dd) (void)hipFree(dd);
    if (ds) (void)hipFree(ds);
    if (dl) (void)hipFree(dl);
  };
  if (hipMalloc((void **)&dd, n * 8) != hipSuccess || hipMalloc((void **)&ds, n * 8) != hipSuccess ||
      hipMalloc((void **)&dl, n * 8) != hipSuccess) {
    (void)hipGetLastError();
    cleanup();
    return fail(BCD_ERR_OUT_OF_MEMORY, "export buffers");
  }
  bool ovf = false;
  ProfAcc prof;
  std::vector<int32_t> none;
  bcd_status rc = run_plain_one(g, ws, s, nullptr, 0, none, true, nullptr, dd, ds, dl, &prof, &ovf);
  if (rc == BCD_OK) {
    hipError_t e = hipSuccess;
    if (dist) e = hipMemcpy(dist, dd, n * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess && sigma) e = hipMemcpy(sigma, ds, n * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess && delta) e = hipMemcpy(delta, dl, n * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = hip_fail(e, "export copy");
  }
  cleanup();
  uint64_t c[C_COUNT];
  if (rc == BCD_OK) rc = collect_counters(ws, c, ws->P.acc);
  if (rc == BCD_OK && ovf) rc = fail(BCD_ERR_SIGMA_OVERFLOW, "a shortest-path count exceeded 2^64 - 1");
  return rc;
  BCD_GUARD_END
}

}  // extern "C"
