// Host-side objects of libbcd: the resident graph and per-call workspaces.
#pragma once

#include <atomic>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/bcd.h"
#include "bcd_internal.h"

// Error propagation inside the host layer.
#define HIPCHK(expr)                                  \
  do {                                                \
    hipError_t _e = (expr);                           \
    if (_e != hipSuccess) return hip_fail(_e, #expr); \
  } while (0)

#define STCHK(expr)              \
  do {                           \
    bcd_status _s = (expr);      \
    if (_s != BCD_OK) return _s; \
  } while (0)

// Body of every exported call: a C++ exception (an allocation failure in
// host code) becomes a status with its message; none crosses the C ABI.
#define BCD_GUARD_BEGIN try {
#define BCD_GUARD_END                                                   \
  }                                                                     \
  catch (const std::bad_alloc &) {                                      \
    return bcd::fail(BCD_ERR_OUT_OF_MEMORY, "host allocation failed"); \
  }                                                                     \
  catch (...) {                                                         \
    return bcd::fail(BCD_ERR_DEVICE, "unexpected host exception");     \
  }

namespace bcd {

constexpr int kCtrSlots = 8192;       // max workgroups of a traversal launch
constexpr int kLevelChunkMax = 64;    // level launches enqueued between host checks
constexpr int kDefaultItems = 2;      // frontier items per wavefront step, unweighted forward
// Bottom-up threshold denominator of the unweighted forward (0: top-down
// only).  Bottom-up levels pay on large graphs (R-MAT 20 and 22, acyclic
// R-MAT 20: +4 to +14 %) and cost a little on small ones (R-MAT 16: -4 %).
inline int default_bottom_up(int64_t n) { return n >= (int64_t(1) << 19) ? 4 : 0; }
// Top-down levels of the unweighted forward add path counts along DAG arcs
// (1) instead of pulling them over in-arcs (0).
constexpr int kDefaultPush = 0;
constexpr int kMaxParts = 8;          // item-list partitions (one per XCD)
constexpr int kCntStage = (kLevelChunkMax + 2) * kMaxParts;  // pinned slots for level counts

bcd_status fail(bcd_status s, const std::string &msg);
bcd_status fail_static(bcd_status s, const char *msg);  // records the message without allocating
bcd_status hip_fail(hipError_t e, const char *what);
bcd_status device_check(int *cus, size_t *lds_block_bytes = nullptr);

inline int default_groups(int64_t n, bool weighted) {
  // keep the [G][n][64] path-count and psi arrays near 64 GiB (HBM is 288 GB),
  // at least one group, at most 96 (128 weighted).  R-MAT 16 runs a query of
  // 33,358 sources in 6 batches of 96 groups 4 % faster than in 9 of 64;
  // wider batches gain nothing more there.  The weighted engine's longer
  // tails favour wider batches: R-MAT 18 weighted 44.6 -> 46.2 GTEPS at 128
  // (46.3 at 192, 41.7 at 256)
  int64_t g = (1ll << 36) / (2 * 8 * 64 * std::max<int64_t>(n, 1));
  if (g < 1) g = 1;
  const int64_t cap = weighted ? 128 : 96;
  if (g > cap) g = cap;
  while (g > 1 && (uint64_t)g * (uint64_t)n >= (1ull << 32)) --g;
  // group j runs in XCD partition j % 8: above 8 groups, a width that is not
  // a multiple of 8 gives some partitions one group more than the others and
  // every level waits for them (R-MAT 22 serving: 9-group batches 252 GTEPS,
  // 8-group batches 301)
  if (g > 8) g -= g % 8;
  return (int)g;
}

struct Graph;

struct Workspace {
  Graph *graph = nullptr;
  int64_t n = 0;
  bool weighted_graph = false;
  hipStream_t stream = nullptr;
  // batched engine
  bool batch_ready = false;
  int G = 0;
  BatchState S{};
  size_t res_cap = 0;
  // every path count of S.sig is zero (after creation, a dense reset or a
  // batch whose counts were pushed and then cleared); a batch that pulls its
  // counts leaves them behind, and a pushing batch needs them zero
  bool sig_zero = false;
  uint32_t *d_items0 = nullptr;
  unsigned long long *d_masks0 = nullptr;
  uint32_t *d_dest0 = nullptr;
  int32_t *d_lane_slot = nullptr;
  uint32_t *h_items0 = nullptr;
  unsigned long long *h_masks0 = nullptr;
  uint32_t *h_dest0 = nullptr;
  uint32_t h_cnt0[8] = {0};  // level-0 items per partition of the staged batch
  double *h_res = nullptr;
  int last_depth = 8;
  // plain engine
  bool plain_ready = false;
  PlainState P{};
  // reachability
  bool reach_ready = false;
  uint32_t *bitmap = nullptr;
  int32_t *rq[2] = {nullptr, nullptr};
  uint32_t *rqn = nullptr;  // [8]: per queue c, length at 4c, arcs of its vertices (uint64) at 4c + 2
  uint32_t *h_bitmap = nullptr;
  // host staging
  uint32_t *h_cnt = nullptr;
  uint64_t *h_misc = nullptr;
  uint64_t *h_ctr = nullptr;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  // server batches: target list and result routes, grown on demand and kept
  // (a free in the batch loop would wait for every stream of the device)
  int32_t *d_tgt_list = nullptr;
  size_t tgt_list_cap = 0;
  ResultRoute *d_routes = nullptr;
  size_t routes_cap = 0;
  bcd_status ensure_server_lists(size_t ntgt, size_t nroutes);
  // LDS engine scratch (bcd_lds.hip), grown on demand
  void *lds_dev = nullptr;
  size_t lds_dev_bytes = 0;
  void *lds_host = nullptr;
  size_t lds_host_bytes = 0;

  ~Workspace();
  void release();
  bcd_status init_common(Graph *g);
  bcd_status ensure_reach();
  bcd_status ensure_batch(int G);
  bcd_status ensure_res(size_t need);
  bcd_status ensure_dout();
  bcd_status grow_items();
  bcd_status reset_batch_dense();
  bcd_status ensure_plain();
  // Stage a batch: lane i of the batch (column group i / 64, lane i % 64)
  // runs source vertex src[i]; vertices must be distinct within a group.
  void stage_sources(const int32_t *src, int k);
  void stage_sources_dest(int k);
  // Partitions a batch of k staged sources uses: its groups are 0..ceil(k/64)-1
  // and group g belongs to partition g % P, so a batch of fewer groups than
  // S.P uses one partition per group and no workgroup is left without work.
  int batch_parts(int k) const { return std::max(1, std::min(S.P, (k + kLanes - 1) / kLanes)); }
  int staged = 0;
  bool weighted_ready = false;
  int weighted_G = 0;
  bcd_status ensure_weighted();
  void release_weighted();
  std::pair<hipEvent_t, hipEvent_t> event_pair(size_t i);
};

struct Graph {
  int64_t n = 0, m = 0;
  bool weighted = false;
  uint32_t max_w = 1;
  int cus = 1;
  size_t lds_block_bytes = 0;  // LDS one workgroup may allocate
  std::vector<int64_t> h_rp;
  // compression (computed on the first compressed call): gate[v] = the vertex
  // every path from v leaves through when v lies on no cycle and all its
  // out-neighbours funnel into that one vertex, else -1
  std::mutex gate_mu;
  bool gates_ready = false;
  std::vector<int32_t> gate;
  int64_t *d_rp = nullptr;
  int32_t *d_col = nullptr;
  int64_t *d_irp = nullptr;
  int32_t *d_icol = nullptr;
  uint2 *d_arcw = nullptr;     // weighted: {head, length} per CSR arc
  uint2 *d_arcp = nullptr;     // weighted: {head, transpose position} per CSR arc
  uint2 *d_iarc = nullptr;     // weighted: {tail, length} per transpose arc
  mutable std::mutex cfg_mu;
  bcd_config cfg{};
  std::mutex pool_mu;
  std::vector<std::unique_ptr<Workspace>> pool;
  std::atomic<bool> profiling{false};
  std::mutex lm_mu;                // landmark distance signatures (source ordering)
  bool lm_ready = false;
  std::vector<uint8_t> lm_sig;     // [n][16] BFS distance to each hub, 255 = unreachable
  mutable std::mutex prof_mu;
  bcd_kernel_profile prof[2]{};
  hipEvent_t prof_ref = nullptr;                      // origin of the launch intervals below
  std::vector<std::pair<double, double>> prof_iv[2];  // launch [start, end], ms after prof_ref
  double prof_solo_ms[2] = {0, 0};                    // launches timed without an interval
  bcd_status mark_profile_origin();

  ~Graph();
  DevGraph dev() const;
  Launch launch() const;
  Launch launch_parts(int P) const;  // grid a multiple of P
  bcd_config config() const;
  std::unique_ptr<Workspace> acquire();
  void release(std::unique_ptr<Workspace> w);
  void trim_pool();  // free the device memory of idle pooled workspaces
  void add_profile(int kind, int64_t launches, double ms, const uint64_t *c3, double alg_bytes,
                   uint64_t items = 0, const std::vector<std::pair<double, double>> *intervals = nullptr,
                   uint64_t item_arcs = 0, double sched_bytes = -1.0);
  int64_t outdeg(int64_t v) const { return h_rp[(size_t)v + 1] - h_rp[(size_t)v]; }
};

// Scoped workspace lease.
struct Lease {
  Graph *g;
  std::unique_ptr<Workspace> w;
  explicit Lease(Graph *g_) : g(g_), w(g_->acquire()) {}
  ~Lease() { g->release(std::move(w)); }
  Workspace *operator->() { return w.get(); }
  bool ok() const { return (bool)w; }
};

// Per-source results of one run over a source list.
struct SourceRun {
  std::vector<double> dep;          // [ns][ntgt]
  std::vector<uint64_t> counters;   // [ns][3] when requested
  uint64_t te = 0, reached = 0, dag = 0;
  int32_t width = 0;
};

struct TargetMap {
  Workspace *ws;
  int32_t *d_verts = nullptr;
  int k = 0;
  bool set = false;
  ~TargetMap() {
    if (set) {
      (void)launch_scatter_targets(ws->S.tgt_of, d_verts, k, 0, ws->stream);
      (void)hipStreamSynchronize(ws->stream);
    }
    if (d_verts) (void)hipFree(d_verts);
  }
  bcd_status install(Workspace *w, const std::vector<int32_t> &tgt) {
    ws = w;
    k = (int)tgt.size();
    if (k == 0) return BCD_OK;
    if (hipMalloc((void **)&d_verts, (size_t)k * sizeof(int32_t)) != hipSuccess) {
      (void)hipGetLastError();
      d_verts = nullptr;
      return fail(BCD_ERR_OUT_OF_MEMORY, "target list allocation failed");
    }
    HIPCHK(hipMemcpyAsync(d_verts, tgt.data(), (size_t)k * sizeof(int32_t), hipMemcpyHostToDevice, ws->stream));
    HIPCHK(launch_scatter_targets(ws->S.tgt_of, d_verts, k, 1, ws->stream));
    set = true;
    return BCD_OK;
  }
};

// Launch timings of one run, per kind (0 forward, 1 backward), gathered while
// the graph's profiling is on.
struct ProfAcc {
  int64_t launches[2] = {0, 0};
  double ms[2] = {0, 0};
  uint64_t items[2] = {0, 0};
  std::vector<std::pair<double, double>> iv[2];  // launch intervals after the graph's profile origin
  void merge(const ProfAcc &o) {
    for (int k = 0; k < 2; ++k) {
      launches[k] += o.launches[k];
      ms[k] += o.ms[k];
      items[k] += o.items[k];
      iv[k].insert(iv[k].end(), o.iv[k].begin(), o.iv[k].end());
    }
  }
  // one launch bracketed by the event pair (a, b)
  void add(const Graph *g, int kind, hipEvent_t a, hipEvent_t b);
};

// Batches b = first, first + stride, ... of one run on workspace `ws`
// (ws's own stream; results to their own positions).
using StripeFn = std::function<bcd_status(Workspace *ws, size_t first, size_t stride, ProfAcc &prof, bool &ovf)>;
// Runs `stripe` over all batches; when the run has more than one batch and a
// second workspace can be had (`prepare` readies it), every other batch goes
// to that workspace on a helper thread.  The second workspace's counters are
// added to `tot`.
bcd_status run_pipelined(Graph *g, Workspace *ws, size_t nbatches, const std::function<bcd_status(Workspace *)> &prepare,
                         const StripeFn &stripe, ProfAcc &prof, bool &ovf, uint64_t *tot);

// Query layer (bcd_query.hip).
bcd_status reach_set(Graph *g, Workspace *ws, int32_t root, bool reverse, std::vector<uint32_t> &bits,
                     int64_t *count, uint8_t *d_lev);
bcd_status run_weighted(Graph *g, Workspace *ws, const std::vector<int32_t> &src,
                        const std::vector<int32_t> &tgt, bool want_counters, SourceRun &out);
bcd_status multi_source_pass_weighted(Graph *g, const int32_t *sources, int64_t k, uint64_t *dist,
                                      uint64_t *sigma, double *delta);
// Device bytes of one batch workspace of `groups` column groups (bcd_server.hip).
uint64_t batch_workspace_bytes(const Graph *g, int groups);
// LDS engine (bcd_lds.hip): one workgroup per source at a time, state in LDS.
size_t lds_bytes_for(int64_t n);
bool lds_fits(const Graph *g);
// Single-workgroup reachability (n < 2^16, visited bits and queue in LDS).
bool lds_reach_fits(const Graph *g);
hipError_t launch_lds_reach(const Graph *g, const int64_t *rp, const int32_t *col, int32_t root, uint32_t *bitmap,
                            hipStream_t st);
bcd_status run_lds(Graph *g, Workspace *ws, const std::vector<int32_t> &src, const std::vector<int32_t> &tgt,
                   bool want_counters, SourceRun &out);
bcd_status multi_source_pass_lds(Graph *g, Workspace *ws, const int32_t *sources, int64_t k, uint64_t *dist,
                                 uint64_t *sigma, double *delta);
// One batch of `k` sources already staged in ws->h_items0 / h_masks0 with
// ntgt targets installed in ws->S.tgt_of; per-lane target dependencies stay
// in ws->S.res on the device; per-group overflow lanes go to ovl_out[G].
// Launch timings go to *prof when the graph's profiling is on (may be NULL).
bcd_status run_staged_batch(Graph *g, Workspace *ws, int k, int ntgt, unsigned long long *ovl_out, bool *ovf,
                            ProfAcc *prof);
bcd_status run_staged_wbatch(Graph *g, Workspace *ws, int k, int ntgt, unsigned long long *ovl_out, bool *ovf,
                             ProfAcc *prof);
// Add one run's launch timings and its device counters to the graph's profile.
void record_profile(Graph *g, const ProfAcc &p, const uint64_t *ctr);
void record_wprofile(Graph *g, const ProfAcc &p, const uint64_t *ctr);
double compensated_sum(const double *x, size_t k, size_t stride);
// Positions of src in the order batches should take them (sources with
// similar hub-distance signatures together); results never depend on it.
bcd_status source_order(Graph *g, Workspace *ws, const std::vector<int32_t> &src, std::vector<uint32_t> &ord);
bcd_status collect_counters(Workspace *ws, uint64_t *ctr, uint64_t *dev_acc);
uint64_t splitmix_at(uint64_t seed, uint64_t t);
uint64_t index_below(uint64_t x, uint64_t k);
void bits_to_list(const std::vector<uint32_t> &bits, int64_t n, int32_t skip, std::vector<int32_t> &out);
bcd_status run_sources(Graph *g, Workspace *ws, const std::vector<int32_t> &src,
                       const std::vector<int32_t> &tgt, bool want_counters, SourceRun &out);

}  // namespace bcd
