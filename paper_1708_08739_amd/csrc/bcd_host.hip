// libbcd host layer: the C ABI of include/bcd.h.
//
// Graph: the out-CSR and its transpose (the reverse graph of Def.2) are
// uploaded once and stay resident.  Queries: RV(r) by a device BFS on the
// transpose (Def.3, Prop.2), then batches of sources through the batched
// forward / backward kernels, then a compensated sum on the host in a fixed
// order (ascending source for Alg.1, draw order for Alg.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/bcd.h"
#include "bcd_internal.h"
#include "bcd_host_internal.h"

namespace bcd {

// Message of the calling thread's last failing call, in a fixed buffer so
// that recording it never allocates.
static thread_local char t_last_error[512];

static void set_last_error(const char *msg, size_t len) {
  if (len >= sizeof(t_last_error)) len = sizeof(t_last_error) - 1;
  std::memcpy(t_last_error, msg, len);
  t_last_error[len] = '\0';
}

bcd_status fail(bcd_status s, const std::string &msg) {
  set_last_error(msg.data(), msg.size());
  return s;
}

bcd_status fail_static(bcd_status s, const char *msg) {
  set_last_error(msg, std::strlen(msg));
  return s;
}

bcd_status hip_fail(hipError_t e, const char *what) {
  return fail(BCD_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}


static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------ device

bcd_status device_check(int *cus, size_t *lds_block_bytes) {
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0) return fail(BCD_ERR_DEVICE, "no HIP device available");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(BCD_ERR_DEVICE, std::string("libbcd is built for gfx950; device is ") + prop.gcnArchName);
  if (cus) *cus = prop.multiProcessorCount;
  if (lds_block_bytes) *lds_block_bytes = prop.sharedMemPerBlock;
  return BCD_OK;
}

template <class T>
static bcd_status dalloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void **)p, count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(BCD_ERR_OUT_OF_MEMORY, std::string("device allocation of ") +
                                           std::to_string(count * sizeof(T)) + " bytes failed");
  }
  return BCD_OK;
}

template <class T>
static bcd_status halloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipHostMalloc((void **)p, count * sizeof(T), hipHostMallocDefault);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(BCD_ERR_OUT_OF_MEMORY, "pinned host allocation failed");
  }
  return BCD_OK;
}

template <class T>
static void dfree(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

template <class T>
static void hfree(T *&p) {
  if (p) (void)hipHostFree((void *)p);
  p = nullptr;
}

// ---------------------------------------------------------- workspace

Workspace::~Workspace() { release(); }

void Workspace::release() {
  release_weighted();
  dfree(d_tgt_list);
  dfree(d_routes);
  tgt_list_cap = routes_cap = 0;
  if (lds_dev) (void)hipFree(lds_dev);
  if (lds_host) (void)hipHostFree(lds_host);
  lds_dev = lds_host = nullptr;
  lds_dev_bytes = lds_host_bytes = 0;
  dfree(S.sig);
  dfree(S.psi);
  dfree(S.dout);
  dfree(S.vis);
  dfree(S.fr);
  dfree(S.rec);
  dfree(S.bt);
  dfree(S.items);
  dfree(S.imask);
  dfree(S.cnt);
  dfree(S.off);
  dfree(S.tmin);
  dfree(S.tgt_of);
  dfree(S.res);
  dfree(S.ctr);
  dfree(S.acc);
  dfree(S.flags);
  dfree(S.ovl);
  dfree(d_items0);
  dfree(d_masks0);
  dfree(d_dest0);
  hfree(h_dest0);
  dfree(d_lane_slot);
  dfree(P.d);
  dfree(P.sig);
  dfree(P.psi);
  dfree(P.dout);
  dfree(P.queue);
  dfree(P.cnt);
  dfree(P.off);
  dfree(P.ctr);
  dfree(P.acc);
  dfree(P.flags);
  dfree(bitmap);
  dfree(rq[0]);
  dfree(rq[1]);
  dfree(rqn);
  hfree(h_items0);
  hfree(h_masks0);
  hfree(h_cnt);
  hfree(h_misc);
  hfree(h_res);
  hfree(h_ctr);
  hfree(h_bitmap);
  for (auto &ev : events) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  events.clear();
  if (stream) (void)hipStreamDestroy(stream);
  stream = nullptr;
  batch_ready = plain_ready = reach_ready = false;
}

bcd_status Workspace::init_common(Graph *g) {
  graph = g;
  n = g->n;
  weighted_graph = g->weighted;
  if (!stream) HIPCHK(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
  return BCD_OK;
}

bcd_status Workspace::ensure_reach() {
  if (reach_ready) return BCD_OK;
  // what an earlier call that failed part way left allocated
  dfree(bitmap); dfree(rq[0]); dfree(rq[1]); dfree(rqn); hfree(h_bitmap);
  const size_t words = (size_t)(n + 31) / 32;
  STCHK(dalloc(&bitmap, words));
  STCHK(dalloc(&rq[0], (size_t)n));
  STCHK(dalloc(&rq[1], (size_t)n));
  STCHK(dalloc(&rqn, 8));  // two queues: length, pad, arcs (uint64)
  STCHK(halloc(&h_bitmap, words));
  if (!h_misc) STCHK(halloc(&h_misc, 64));  // shared with the plain engine
  reach_ready = true;
  return BCD_OK;
}

bcd_status Workspace::ensure_batch(int G_) {
  if (batch_ready && G == G_) return BCD_OK;
  // the previous width's arrays, or what an earlier call that failed part
  // way left allocated (every free is a no-op on a null pointer)
  release_weighted();
  dfree(S.sig); dfree(S.psi); dfree(S.dout); dfree(S.vis); dfree(S.fr); dfree(S.rec); dfree(S.bt);
  dfree(S.items); dfree(S.imask); dfree(S.cnt); dfree(S.off); dfree(S.tmin);
  dfree(S.tgt_of); dfree(S.res); dfree(S.ctr); dfree(S.acc); dfree(S.flags); dfree(S.ovl);
  dfree(d_items0); dfree(d_masks0); dfree(d_dest0); dfree(d_lane_slot); hfree(h_items0); hfree(h_masks0);
  hfree(h_dest0); hfree(h_res);
  res_cap = 0;
  batch_ready = false;
  if ((uint64_t)G_ * (uint64_t)n >= (1ull << 32))
    return fail(BCD_ERR_UNSUPPORTED, "groups * n must stay below 2^32");
  G = G_;
  const size_t GN = (size_t)G * (size_t)n;
  std::memset(&S, 0, sizeof(S));
  S.n = n;
  S.G = G;
  STCHK(dalloc(&S.sig, GN * kLanes));
  STCHK(dalloc(&S.psi, GN * kLanes));
  if (weighted_graph) {
    STCHK(dalloc(&S.vis, GN));
    STCHK(dalloc(&S.fr, 3 * GN));
  } else {
    STCHK(dalloc(&S.rec, GN));
  }
  STCHK(dalloc(&S.bt, 2 * GN));
  S.P = std::min(kMaxParts, G);
  S.capP = ((uint64_t)GN * 16 + (uint64_t)S.P - 1) / (uint64_t)S.P;
  S.cap = S.capP * (uint64_t)S.P;
  STCHK(dalloc(&S.items, S.cap));
  STCHK(dalloc(&S.imask, S.cap));
  const size_t levels = ((size_t)n + kLevelChunkMax + 4) * kMaxParts;
  STCHK(dalloc(&S.cnt, levels));
  STCHK(dalloc(&S.off, levels));
  STCHK(dalloc(&S.tmin, 4));
  STCHK(dalloc(&S.tgt_of, (size_t)n));
  STCHK(dalloc(&S.flags, 4));
  STCHK(dalloc(&S.ovl, (size_t)G));
  S.ctr_slots = kCtrSlots;
  STCHK(dalloc(&S.ctr, (size_t)kCtrSlots * C_COUNT));
  STCHK(dalloc(&S.acc, (size_t)C_COUNT));
  HIPCHK(hipMemsetAsync(S.acc, 0, (size_t)C_COUNT * sizeof(uint64_t), stream));
  res_cap = (size_t)G * kLanes;
  STCHK(dalloc(&S.res, res_cap));
  STCHK(dalloc(&d_items0, (size_t)G * kLanes));
  STCHK(dalloc(&d_masks0, (size_t)G * kLanes));
  STCHK(dalloc(&d_dest0, (size_t)G * kLanes));
  STCHK(halloc(&h_dest0, (size_t)G * kLanes));
  STCHK(dalloc(&d_lane_slot, (size_t)G * kLanes));
  STCHK(halloc(&h_items0, (size_t)G * kLanes));
  STCHK(halloc(&h_masks0, (size_t)G * kLanes));
  STCHK(halloc(&h_res, res_cap));
  if (!h_cnt) STCHK(halloc(&h_cnt, kCntStage + 16));
  if (!h_misc) STCHK(halloc(&h_misc, 64));
  if (!h_ctr) STCHK(halloc(&h_ctr, (size_t)kCtrSlots * C_COUNT));
  HIPCHK(hipMemsetAsync(S.sig, 0, GN * kLanes * sizeof(uint64_t), stream));
  if (S.vis) HIPCHK(hipMemsetAsync(S.vis, 0, GN * sizeof(uint64_t), stream));
  if (S.fr) HIPCHK(hipMemsetAsync(S.fr, 0, 3 * GN * sizeof(uint64_t), stream));
  if (S.rec) HIPCHK(hipMemsetAsync(S.rec, 0, GN * sizeof(MaskRec), stream));
  HIPCHK(hipMemsetAsync(S.bt, 0, 2 * GN * sizeof(LevMask), stream));
  HIPCHK(hipMemsetAsync(S.cnt, 0, levels * sizeof(uint32_t), stream));
  HIPCHK(hipMemsetAsync(S.off, 0, levels * sizeof(uint64_t), stream));
  HIPCHK(hipMemsetAsync(S.tgt_of, 0xFF, (size_t)n * sizeof(int32_t), stream));
  HIPCHK(hipMemsetAsync(S.flags, 0, 4 * sizeof(uint32_t), stream));
  HIPCHK(hipMemsetAsync(S.ctr, 0, (size_t)kCtrSlots * C_COUNT * sizeof(uint64_t), stream));
  HIPCHK(hipStreamSynchronize(stream));
  S.epoch = 0;
  sig_zero = true;
  batch_ready = true;
  return BCD_OK;
}


void Workspace::stage_sources(const int32_t *src, int k) {
  for (int i = 0; i < k; ++i) {
    h_items0[i] = (uint32_t)((uint64_t)(i / kLanes) * (uint64_t)n + (uint64_t)src[i]);
    h_masks0[i] = 1ull << (i % kLanes);
  }
  staged = k;
  stage_sources_dest(k);
}

// Level-0 slot of every staged item in its group's partition.
void Workspace::stage_sources_dest(int k) {
  uint32_t fill[kMaxParts] = {0};
  const int P = batch_parts(k);
  for (int i = 0; i < k; ++i) {
    const int p = (i / kLanes) % P;
    h_dest0[i] = (uint32_t)((uint64_t)p * S.capP + fill[p]++);
  }
  for (int p = 0; p < kMaxParts; ++p) h_cnt0[p] = fill[p];
}

bcd_status Workspace::ensure_res(size_t need) {
  if (need <= res_cap) return BCD_OK;
  dfree(S.res);
  hfree(h_res);
  res_cap = 0;  // recorded only once both buffers exist
  STCHK(dalloc(&S.res, need));
  STCHK(halloc(&h_res, need));
  res_cap = need;
  return BCD_OK;
}

bcd_status Workspace::ensure_server_lists(size_t ntgt, size_t nroutes) {
  ntgt = std::max<size_t>(ntgt, 1);
  nroutes = std::max<size_t>(nroutes, 1);
  if (ntgt > tgt_list_cap) {
    const size_t cap = std::max<size_t>(ntgt, 2 * tgt_list_cap + 64);
    dfree(d_tgt_list);
    tgt_list_cap = 0;
    STCHK(dalloc(&d_tgt_list, cap));
    tgt_list_cap = cap;
  }
  if (nroutes > routes_cap) {
    const size_t cap = std::max<size_t>(nroutes, 2 * routes_cap + 1024);
    dfree(d_routes);
    routes_cap = 0;
    STCHK(dalloc(&d_routes, cap));
    routes_cap = cap;
  }
  return BCD_OK;
}

bcd_status Workspace::ensure_dout() {
  if (S.dout) return BCD_OK;
  return dalloc(&S.dout, (size_t)G * (size_t)n * kLanes);
}

bcd_status Workspace::grow_items() {
  const uint64_t GN = (uint64_t)G * (uint64_t)n;
  const uint64_t ncapP = std::min<uint64_t>(S.capP * 2, (GN * kLanes) / (uint64_t)S.P + (uint64_t)kLanes * G);
  dfree(S.items);
  dfree(S.imask);
  S.capP = ncapP;
  S.cap = S.capP * (uint64_t)S.P;
  // if an allocation fails the workspace must not be reused as it stands:
  // the next ensure_batch rebuilds every array
  batch_ready = false;
  STCHK(dalloc(&S.items, S.cap));
  STCHK(dalloc(&S.imask, S.cap));
  batch_ready = true;
  return BCD_OK;
}

// Full reset after an aborted batch (item list overflow, or a host exception
// in a server worker): the sparse cleanup cannot see items that were never
// stored.
bcd_status Workspace::reset_batch_dense() {
  const size_t GN = (size_t)G * (size_t)n;
  HIPCHK(hipMemsetAsync(S.sig, 0, GN * kLanes * sizeof(uint64_t), stream));
  sig_zero = true;
  if (S.vis) HIPCHK(hipMemsetAsync(S.vis, 0, GN * sizeof(uint64_t), stream));
  if (S.fr) HIPCHK(hipMemsetAsync(S.fr, 0, 3 * GN * sizeof(uint64_t), stream));
  if (S.rec) HIPCHK(hipMemsetAsync(S.rec, 0, GN * sizeof(MaskRec), stream));
  HIPCHK(hipMemsetAsync(S.cnt, 0, ((size_t)n + kLevelChunkMax + 4) * kMaxParts * sizeof(uint32_t), stream));
  HIPCHK(hipMemsetAsync(S.flags, 0, 4 * sizeof(uint32_t), stream));
  HIPCHK(hipMemsetAsync(S.ctr, 0, (size_t)kCtrSlots * C_COUNT * sizeof(uint64_t), stream));
  if (weighted_ready) {
    HIPCHK(hipMemsetAsync(S.wd, 0xFF, GN * kLanes * sizeof(uint32_t), stream));
    HIPCHK(hipMemsetAsync(S.wc, 0, GN * kLanes * sizeof(uint32_t), stream));
    HIPCHK(hipMemsetAsync(S.chg, 0, 2 * GN * sizeof(unsigned long long), stream));
    HIPCHK(hipMemsetAsync(S.bqn, 0, 4 * sizeof(uint32_t), stream));
    HIPCHK(hipMemsetAsync(S.rln, 0, sizeof(uint32_t), stream));
    HIPCHK(hipMemsetAsync(S.wdn, 0, GN * sizeof(unsigned long long), stream));
  }
  HIPCHK(hipStreamSynchronize(stream));
  return BCD_OK;
}

bcd_status Workspace::ensure_plain() {
  if (plain_ready) return BCD_OK;
  // what an earlier call that failed part way left allocated
  dfree(P.d); dfree(P.sig); dfree(P.psi); dfree(P.dout); dfree(P.queue);
  dfree(P.cnt); dfree(P.off); dfree(P.flags); dfree(P.ctr); dfree(P.acc);
  std::memset(&P, 0, sizeof(P));
  P.n = n;
  STCHK(dalloc(&P.d, (size_t)n));
  STCHK(dalloc(&P.sig, (size_t)n));
  STCHK(dalloc(&P.psi, (size_t)n));
  STCHK(dalloc(&P.dout, (size_t)n));
  STCHK(dalloc(&P.queue, (size_t)n));
  const size_t levels = (size_t)n + kLevelChunkMax + 4;
  STCHK(dalloc(&P.cnt, levels));
  STCHK(dalloc(&P.off, levels));
  STCHK(dalloc(&P.flags, 4));
  P.ctr_slots = kCtrSlots;
  STCHK(dalloc(&P.ctr, (size_t)kCtrSlots * C_COUNT));
  STCHK(dalloc(&P.acc, (size_t)C_COUNT));
  HIPCHK(hipMemsetAsync(P.acc, 0, (size_t)C_COUNT * sizeof(uint64_t), stream));
  if (!h_cnt) STCHK(halloc(&h_cnt, kCntStage + 16));
  if (!h_misc) STCHK(halloc(&h_misc, 64));
  if (!h_ctr) STCHK(halloc(&h_ctr, (size_t)kCtrSlots * C_COUNT));
  HIPCHK(hipMemsetAsync(P.d, 0xFF, (size_t)n * sizeof(int32_t), stream));
  HIPCHK(hipMemsetAsync(P.sig, 0, (size_t)n * sizeof(uint64_t), stream));
  HIPCHK(hipMemsetAsync(P.cnt, 0, levels * sizeof(uint32_t), stream));
  HIPCHK(hipMemsetAsync(P.off, 0, levels * sizeof(uint64_t), stream));
  HIPCHK(hipMemsetAsync(P.flags, 0, 4 * sizeof(uint32_t), stream));
  HIPCHK(hipMemsetAsync(P.ctr, 0, (size_t)kCtrSlots * C_COUNT * sizeof(uint64_t), stream));
  HIPCHK(hipStreamSynchronize(stream));
  plain_ready = true;
  return BCD_OK;
}

std::pair<hipEvent_t, hipEvent_t> Workspace::event_pair(size_t i) {
  while (events.size() <= i) {
    hipEvent_t a = nullptr, b = nullptr;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    events.emplace_back(a, b);
  }
  return events[i];
}

// ------------------------------------------------------------- graph

Graph::~Graph() {
  pool.clear();
  if (prof_ref) (void)hipEventDestroy(prof_ref);
  dfree(d_rp);
  dfree(d_col);
  dfree(d_irp);
  dfree(d_icol);
  dfree(d_arcw);
  dfree(d_arcp);
  dfree(d_iarc);
}

DevGraph Graph::dev() const {
  DevGraph G;
  G.n = n;
  G.m = m;
  G.rp = d_rp;
  G.col = d_col;
  G.irp = d_irp;
  G.icol = d_icol;
  G.arcw = d_arcw;
  G.arcp = d_arcp;
  G.iarc = d_iarc;
  return G;
}

Launch Graph::launch_parts(int P) const {
  Launch L = launch();
  if (P > 1) L.grid = std::max(P, L.grid - L.grid % P);
  return L;
}

Launch Graph::launch() const {
  Launch L;
  std::lock_guard<std::mutex> lk(cfg_mu);
  L.block = cfg.block;
  L.grid = std::max(1, std::min(kCtrSlots, cus * cfg.grid_mult));
  L.items = cfg.items;
  return L;
}

bcd_config Graph::config() const {
  std::lock_guard<std::mutex> lk(cfg_mu);
  return cfg;
}

void Graph::trim_pool() {
  std::vector<std::unique_ptr<Workspace>> idle;
  {
    std::lock_guard<std::mutex> lk(pool_mu);
    idle.swap(pool);
  }
  // destroyed here, outside the lock
}

std::unique_ptr<Workspace> Graph::acquire() {
  {
    std::lock_guard<std::mutex> lk(pool_mu);
    if (!pool.empty()) {
      std::unique_ptr<Workspace> w = std::move(pool.back());
      pool.pop_back();
      return w;
    }
  }
  std::unique_ptr<Workspace> w(new (std::nothrow) Workspace());
  return w;
}

void Graph::release(std::unique_ptr<Workspace> w) {
  if (!w) return;
  std::lock_guard<std::mutex> lk(pool_mu);
  pool.push_back(std::move(w));
}

bcd_status Graph::mark_profile_origin() {
  if (!prof_ref) HIPCHK(hipEventCreate(&prof_ref));
  HIPCHK(hipEventRecord(prof_ref, nullptr));
  HIPCHK(hipEventSynchronize(prof_ref));
  return BCD_OK;
}

void Graph::add_profile(int kind, int64_t launches, double ms, const uint64_t *c3, double alg_bytes,
                        uint64_t items, const std::vector<std::pair<double, double>> *intervals,
                        uint64_t item_arcs, double sched_bytes) {
  std::lock_guard<std::mutex> lk(prof_mu);
  bcd_kernel_profile &p = prof[kind];
  p.launches += launches;
  p.total_ms += ms;
  p.alg_bytes += alg_bytes;
  p.item_arcs += item_arcs;
  p.sched_bytes += sched_bytes < 0 ? alg_bytes : sched_bytes;
  p.vertex_pairs += c3[0];
  p.arc_pairs += c3[1];
  p.dag_pairs += c3[2];
  p.items += items;
  if (intervals && !intervals->empty())
    prof_iv[kind].insert(prof_iv[kind].end(), intervals->begin(), intervals->end());
  else
    prof_solo_ms[kind] += ms;
}

}  // namespace bcd

using namespace bcd;

// ----------------------------------------------------------------- ABI

extern "C" {

const char *bcd_status_string(bcd_status s) {
  switch (s) {
    case BCD_OK: return "ok";
    case BCD_ERR_INVALID_ARG: return "invalid argument";
    case BCD_ERR_BAD_GRAPH: return "malformed graph";
    case BCD_ERR_SIGMA_OVERFLOW: return "shortest-path count overflows uint64";
    case BCD_ERR_OUT_OF_MEMORY: return "out of memory";
    case BCD_ERR_DEVICE: return "device error";
    case BCD_ERR_BUFFER_TOO_SMALL: return "buffer too small";
    case BCD_ERR_UNSUPPORTED: return "unsupported";
    case BCD_ERR_AGAIN: return "try again";
    case BCD_ERR_CANCELLED: return "cancelled";
  }
  return "unknown status";
}

const char *bcd_last_error(void) { return t_last_error; }

bcd_status bcd_sample_count(double eps_abs, double delta, double K, int64_t rv_size, int64_t *T) {
  BCD_GUARD_BEGIN
  if (!T) return fail(BCD_ERR_INVALID_ARG, "T is NULL");
  if (!(eps_abs > 0.0) || !std::isfinite(eps_abs)) return fail(BCD_ERR_INVALID_ARG, "eps must be > 0");
  if (!(delta > 0.0 && delta < 1.0)) return fail(BCD_ERR_INVALID_ARG, "delta must be in (0,1)");
  if (!(K >= 0.0) || !std::isfinite(K)) return fail(BCD_ERR_INVALID_ARG, "K must be >= 0");
  if (rv_size < 0) return fail(BCD_ERR_INVALID_ARG, "rv_size must be >= 0");
  // Eq.(8), evaluated in extended precision so that ceil is exact for the
  // integer-valued cases; at least one draw.
  const long double x = std::log(2.0L / (long double)delta) * (long double)K * (long double)K *
                        (long double)rv_size * (long double)rv_size /
                        (2.0L * (long double)eps_abs * (long double)eps_abs);
  long double c = std::ceil(x);
  if (!(c >= 1.0L)) c = 1.0L;
  *T = (c >= 9.2e18L) ? INT64_MAX : (int64_t)c;
  return BCD_OK;
  BCD_GUARD_END
}

bcd_status bcd_graph_load_csr(int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col,
                              const uint32_t *weight, bcd_graph **out) {
  BCD_GUARD_BEGIN
  if (!out) return fail(BCD_ERR_INVALID_ARG, "out is NULL");
  if (n <= 0 || n >= (1ll << 31)) return fail(BCD_ERR_INVALID_ARG, "n must be in [1, 2^31)");
  if (m < 0 || m >= (1ll << 32)) return fail(BCD_ERR_INVALID_ARG, "m must be in [0, 2^32)");
  if (!row_ptr || (m > 0 && !col)) return fail(BCD_ERR_INVALID_ARG, "row_ptr/col is NULL");
  // Section 2 graph model: validate fully on the host before touching the GPU.
  if (row_ptr[0] != 0) return fail(BCD_ERR_BAD_GRAPH, "row_ptr[0] != 0");
  if (row_ptr[n] != m) return fail(BCD_ERR_BAD_GRAPH, "row_ptr[n] != m");
  uint64_t max_w = 1;
  for (int64_t v = 0; v < n; ++v) {
    const int64_t a = row_ptr[v], b = row_ptr[v + 1];
    if (b < a) return fail(BCD_ERR_BAD_GRAPH, "row_ptr decreases at vertex " + std::to_string(v));
    if (a < 0 || b > m) return fail(BCD_ERR_BAD_GRAPH, "row_ptr out of [0, m]");
    for (int64_t e = a; e < b; ++e) {
      const int32_t w = col[e];
      if (w < 0 || w >= n) return fail(BCD_ERR_BAD_GRAPH, "column out of range at arc " + std::to_string(e));
      if (w == v) return fail(BCD_ERR_BAD_GRAPH, "self-loop at vertex " + std::to_string(v));
      if (e > a && w <= col[e - 1])
        return fail(BCD_ERR_BAD_GRAPH, "row " + std::to_string(v) + " not strictly increasing (repeated arc?)");
      if (weight) {
        if (weight[e] == 0) return fail(BCD_ERR_BAD_GRAPH, "zero weight at arc " + std::to_string(e));
        max_w = std::max<uint64_t>(max_w, weight[e]);
      }
    }
  }
  int cus = 0;
  size_t lds_block = 0;
  STCHK(device_check(&cus, &lds_block));
  std::unique_ptr<Graph> g(new (std::nothrow) Graph());
  if (!g) return fail(BCD_ERR_OUT_OF_MEMORY, "host allocation failed");
  g->n = n;
  g->m = m;
  g->weighted = weight != nullptr;
  g->max_w = (uint32_t)max_w;
  g->cus = cus;
  g->lds_block_bytes = lds_block;
  g->h_rp.assign(row_ptr, row_ptr + n + 1);
  // transpose by counting sort: rows of R(G) come out sorted
  std::vector<int64_t> irp((size_t)n + 1, 0);
  for (int64_t e = 0; e < m; ++e) irp[(size_t)col[e] + 1]++;
  for (int64_t v = 0; v < n; ++v) irp[(size_t)v + 1] += irp[(size_t)v];
  std::vector<int32_t> icol((size_t)std::max<int64_t>(m, 1));
  std::vector<uint32_t> iw(weight ? (size_t)std::max<int64_t>(m, 1) : 0);
  std::vector<uint32_t> ipos(weight ? (size_t)std::max<int64_t>(m, 1) : 0);
  {
    std::vector<int64_t> fill(irp.begin(), irp.end() - 1);
    for (int64_t u = 0; u < n; ++u)
      for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
        const int64_t p = fill[(size_t)col[e]]++;
        icol[(size_t)p] = (int32_t)u;
        if (weight) {
          iw[(size_t)p] = weight[e];
          ipos[(size_t)e] = (uint32_t)p;
        }
      }
  }
  STCHK(dalloc(&g->d_rp, (size_t)n + 1));
  STCHK(dalloc(&g->d_col, (size_t)m));
  STCHK(dalloc(&g->d_irp, (size_t)n + 1));
  STCHK(dalloc(&g->d_icol, (size_t)m));
  HIPCHK(hipMemcpy(g->d_rp, row_ptr, ((size_t)n + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(g->d_irp, irp.data(), ((size_t)n + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
  if (m > 0) {
    HIPCHK(hipMemcpy(g->d_col, col, (size_t)m * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->d_icol, icol.data(), (size_t)m * sizeof(int32_t), hipMemcpyHostToDevice));
  }
  if (weight) {
    STCHK(dalloc(&g->d_arcw, (size_t)m));
    STCHK(dalloc(&g->d_arcp, (size_t)m));
    STCHK(dalloc(&g->d_iarc, (size_t)m));
    if (m > 0) {
      std::vector<uint2> arcw((size_t)m), arcp((size_t)m);
      std::vector<uint2> iarc((size_t)m);
      for (int64_t e = 0; e < m; ++e) {
        arcw[(size_t)e] = make_uint2((uint32_t)col[e], weight[e]);
        arcp[(size_t)e] = make_uint2((uint32_t)col[e], ipos[(size_t)e]);
        iarc[(size_t)e] = make_uint2((uint32_t)icol[(size_t)e], iw[(size_t)e]);
      }
      HIPCHK(hipMemcpy(g->d_arcw, arcw.data(), (size_t)m * sizeof(uint2), hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(g->d_arcp, arcp.data(), (size_t)m * sizeof(uint2), hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(g->d_iarc, iarc.data(), (size_t)m * sizeof(uint2), hipMemcpyHostToDevice));
    }
  }
  g->cfg.engine = BCD_ENGINE_BATCHED;
  g->cfg.groups = default_groups(n, weight != nullptr);
  // weighted kernels: one-wavefront workgroups, one resident grid (8 waves
  // per SIMD) -- 12 % faster than 256-thread blocks at R-MAT 18
  g->cfg.block = weight ? 64 : 256;
  g->cfg.grid_mult = 32;
  g->cfg.items = kDefaultItems;
  g->cfg.bottom_up = default_bottom_up(n);
  g->cfg.push = kDefaultPush;
  *out = reinterpret_cast<bcd_graph *>(g.release());
  return BCD_OK;
  BCD_GUARD_END
}

bcd_status bcd_graph_free(bcd_graph *g) {
  BCD_GUARD_BEGIN
  if (!g) return BCD_OK;
  delete reinterpret_cast<Graph *>(g);
  return BCD_OK;
  BCD_GUARD_END
}

bcd_status bcd_graph_info(const bcd_graph *gh, int64_t *n, int64_t *m, int32_t *weighted) {
  BCD_GUARD_BEGIN
  if (!gh) return fail(BCD_ERR_INVALID_ARG, "graph is NULL");
  const Graph *g = reinterpret_cast<const Graph *>(gh);
  if (n) *n = g->n;
  if (m) *m = g->m;
  if (weighted) *weighted = g->weighted ? 1 : 0;
  return BCD_OK;
  BCD_GUARD_END
}

bcd_status bcd_set_config(bcd_graph *gh, const bcd_config *cfg) {
  BCD_GUARD_BEGIN
  if (!gh || !cfg) return fail(BCD_ERR_INVALID_ARG, "NULL argument");
  Graph *g = reinterpret_cast<Graph *>(gh);
  if (cfg->engine != BCD_ENGINE_BATCHED && cfg->engine != BCD_ENGINE_PLAIN && cfg->engine != BCD_ENGINE_LDS)
    return fail(BCD_ERR_INVALID_ARG, "unknown engine");
  if (cfg->groups < 1 || (uint64_t)cfg->groups * (uint64_t)g->n >= (1ull << 32))
    return fail(BCD_ERR_INVALID_ARG, "groups must be >= 1 with groups * n < 2^32");
  if (cfg->block != 64 && cfg->block != 128 && cfg->block != 256 && cfg->block != 512)
    return fail(BCD_ERR_INVALID_ARG, "block must be 64, 128, 256 or 512");
  if (cfg->grid_mult < 1 || cfg->grid_mult > 32) return fail(BCD_ERR_INVALID_ARG, "grid_mult must be in [1, 32]");
  if (cfg->items != 0 && cfg->items != 1 && cfg->items != 2 && cfg->items != 4)
    return fail(BCD_ERR_INVALID_ARG, "items must be 1, 2 or 4 (0 = default)");
  if (cfg->bottom_up < -1 || cfg->bottom_up > 4096)
    return fail(BCD_ERR_INVALID_ARG, "bottom_up must be in [-1, 4096]");
  if (cfg->compress != 0 && cfg->compress != 1) return fail(BCD_ERR_INVALID_ARG, "compress must be 0 or 1");
  if (cfg->push < -1 || cfg->push > 1) return fail(BCD_ERR_INVALID_ARG, "push must be -1, 0 or 1");
  std::lock_guard<std::mutex> lk(g->cfg_mu);
  g->cfg = *cfg;
  if (g->cfg.items == 0) g->cfg.items = kDefaultItems;
  if (g->cfg.bottom_up < 0) g->cfg.bottom_up = default_bottom_up(g->n);
  if (g->cfg.push < 0) g->cfg.push = kDefaultPush;
  return BCD_OK;
  BCD_GUARD_END
}

bcd_status bcd_get_config(const bcd_graph *gh, bcd_config *cfg) {
  BCD_GUARD_BEGIN
  if (!gh || !cfg) return fail(BCD_ERR_INVALID_ARG, "NULL argument");
  *cfg = reinterpret_cast<const Graph *>(gh)->config();
  return BCD_OK;
  BCD_GUARD_END
}

bcd_status bcd_profile_enable(bcd_graph *gh, int32_t on) {
  BCD_GUARD_BEGIN
  if (!gh) return fail(BCD_ERR_INVALID_ARG, "graph is NULL");
  Graph *g = reinterpret_cast<Graph *>(gh);
  if (on) {
    std::lock_guard<std::mutex> lk(g->prof_mu);
    STCHK(g->mark_profile_origin());
  }
  g->profiling.store(on != 0);
  return BCD_OK;
  BCD_GUARD_END
}

bcd_status bcd_profile_get(const bcd_graph *gh, int32_t kind, bcd_kernel_profile *out) {
  BCD_GUARD_BEGIN
  if (!gh || !out || kind < 0 || kind > 1) return fail(BCD_ERR_INVALID_ARG, "bad argument");
  const Graph *g = reinterpret_cast<const Graph *>(gh);
  std::lock_guard<std::mutex> lk(g->prof_mu);
  *out = g->prof[kind];
  // measure of the union of the launch intervals (sweep over sorted starts)
  std::vector<std::pair<double, double>> iv = g->prof_iv[kind];
  std::sort(iv.begin(), iv.end());
  double u = 0.0, a = 0.0, b = -1.0;
  bool open = false;
  for (const auto &x : iv) {
    if (!open || x.first > b) {
      if (open) u += b - a;
      a = x.first;
      b = x.second;
      open = true;
    } else {
      b = std::max(b, x.second);
    }
  }
  if (open) u += b - a;
  out->union_ms = u + g->prof_solo_ms[kind];
  return BCD_OK;
  BCD_GUARD_END
}

bcd_status bcd_profile_reset(bcd_graph *gh) {
  BCD_GUARD_BEGIN
  if (!gh) return fail(BCD_ERR_INVALID_ARG, "graph is NULL");
  Graph *g = reinterpret_cast<Graph *>(gh);
  std::lock_guard<std::mutex> lk(g->prof_mu);
  std::memset(g->prof, 0, sizeof(g->prof));
  for (int k = 0; k < 2; ++k) {
    g->prof_iv[k].clear();
    g->prof_solo_ms[k] = 0.0;
  }
  if (g->profiling.load()) STCHK(g->mark_profile_origin());
  return BCD_OK;
  BCD_GUARD_END
}

// Best-of-reps bandwidth of a copy (read = false: `bytes` read and `bytes`
// written per launch) or a read (`bytes` read per launch) over 16-byte words,
// 64 workgroups of 256 threads per compute unit, after one untimed launch.
static bcd_status stream_probe(int64_t bytes, int32_t reps, bool read, double *gbps) {
  if (bytes < 1024 || reps < 1 || !gbps) return fail(BCD_ERR_INVALID_ARG, "bad argument");
  int cus = 0;
  STCHK(device_check(&cus));
  const int64_t n16 = bytes / 16;
  const int grid = std::max(1, cus) * 64;
  uint8_t *a = nullptr, *b = nullptr;
  unsigned *sink = nullptr;
  STCHK(dalloc(&a, (size_t)n16 * 16));
  bcd_status rc = read ? dalloc(&sink, 4) : dalloc(&b, (size_t)n16 * 16);
  if (rc != BCD_OK) {
    dfree(a);
    return rc;
  }
  hipStream_t st;
  hipEvent_t e0, e1;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
    dfree(a);
    dfree(b);
    dfree(sink);
    return fail(BCD_ERR_DEVICE, "stream create failed");
  }
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  (void)hipMemsetAsync(a, 1, (size_t)n16 * 16, st);
  double best = 0;
  const double moved = (read ? 1.0 : 2.0) * (double)n16 * 16;
  for (int i = 0; i < reps + 1 && rc == BCD_OK; ++i) {
    (void)hipEventRecord(e0, st);
    const hipError_t e = read ? launch_read_probe(a, n16, sink, grid, st) : launch_copy_probe(a, b, n16, grid, st);
    if (e != hipSuccess) rc = fail(BCD_ERR_DEVICE, "probe launch failed");
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) rc = fail(BCD_ERR_DEVICE, "probe failed");
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (i > 0 && ms > 0) best = std::max(best, moved / (ms * 1e-3) / 1e9);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(st);
  dfree(a);
  dfree(b);
  dfree(sink);
  if (rc == BCD_OK) *gbps = best;
  return rc;
}

bcd_status bcd_bandwidth_probe(int64_t bytes, int32_t reps, double *gbps) {
  BCD_GUARD_BEGIN
  return stream_probe(bytes, reps, false, gbps);
  BCD_GUARD_END
}

bcd_status bcd_read_bandwidth_probe(int64_t bytes, int32_t reps, double *gbps) {
  BCD_GUARD_BEGIN
  return stream_probe(bytes, reps, true, gbps);
  BCD_GUARD_END
}

}  // extern "C"
