// Small unweighted graphs: the whole per-source pass of one source -- the
// BFS with path counts, then the Eq.(4) accumulation (Alg.1, E-BCD) -- runs
// inside one workgroup with that source's state in LDS.  A source then
// costs one pass over its levels separated by workgroup barriers, instead
// of a kernel launch per level, and all of its state traffic stays on chip
// (the graph itself is read from L2).  Workgroups take sources in turn, so
// one launch serves a whole source list.
//
// LDS per workgroup, for n vertices: sigma u64[n] (overwritten in place by
// psi f64[n] in the backward: psi(v) is written only after sigma(v) has been
// read, and only successors' psi are read), level u32[n], the BFS queue
// u16[n] (vertices in level order) and the level starts u16[n + 2]: 16 n
// bytes plus a little, so n is bounded by what one workgroup may allocate
// (and below 2^16).  Sharing the sigma and psi words lets a CU hold five
// workgroups of a 2,000-vertex graph instead of three.
//
// The graph stays in global memory (it is small enough to sit in L2): a
// copy into each workgroup's LDS was measured slower, since it halves the
// workgroups a CU can hold.
//
// Results are the same bit for bit as the batched engine's: path counts are
// exact integers, and psi(v) = 1/sigma(v) + sum of psi over the DAG
// successors is summed in out-arc order with the same formulas.
//
// The same file holds the single-workgroup reachability kernel used for
// RV(r) (Def.3) on graphs below 2^16 vertices: one launch instead of one
// per BFS level.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/bcd.h"
#include "bcd_device.h"
#include "bcd_host_internal.h"

namespace bcd {

constexpr uint32_t kUnseen = 0xFFFFFFFFu;
constexpr int kLdsBlock = 256;

size_t lds_bytes_for(int64_t n) { return (size_t)16 * (size_t)n + 64; }

bool lds_fits(const Graph *g) {
  return !g->weighted && g->n >= 1 && g->n < 65536 && lds_bytes_for(g->n) <= g->lds_block_bytes;
}

struct LdsArgs {
  const int32_t *src;       // [k] sources
  int k;
  const int32_t *tgt_of;    // [n] target index of a vertex, -1 if none (may be null when ntgt == 0)
  int ntgt;
  int full;                 // backward down to level 0 (for the exports)
  double *res;              // [k][ntgt] delta_s(target)
  uint64_t *cnt;            // [k][3] n_s, m_s, a_s
  uint32_t *ovf;            // [k] 1 if a path count exceeded 2^64 - 1
  uint64_t *xdist;          // [k][n] exports (full only), or null
  unsigned long long *xsig;
  double *xdel;             // [k][n]; entries of unreached vertices are left as they are
};

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_lds_pass(DevGraph G, LdsArgs A) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t n = (uint32_t)G.n;
  // sigma, then (from the backward on) the bits of psi: one array of words,
  // so no two pointer types alias
  ull *sig = reinterpret_cast<ull *>(smem);
  uint32_t *dist = reinterpret_cast<uint32_t *>(smem + 8 * (size_t)n);
  uint16_t *queue = reinterpret_cast<uint16_t *>(smem + 12 * (size_t)n);
  uint16_t *lstart = reinterpret_cast<uint16_t *>(smem + 14 * (size_t)n);  // [n + 2]
  __shared__ uint32_t s_tail, s_ovf, s_stop;
  __shared__ unsigned long long s_m, s_a;
  const uint32_t tid = threadIdx.x;
  for (int i = blockIdx.x; i < A.k; i += gridDim.x) {
    const uint32_t s = (uint32_t)A.src[i];
    for (uint32_t v = tid; v < n; v += BLOCK) {
      dist[v] = kUnseen;
      sig[v] = 0ull;
    }
    for (int t = (int)tid; t < A.ntgt; t += BLOCK) A.res[(size_t)i * A.ntgt + t] = 0.0;
    __syncthreads();
    if (tid == 0) {
      dist[s] = 0u;
      sig[s] = 1ull;
      queue[0] = (uint16_t)s;
      lstart[0] = 0;
      lstart[1] = 1;
      s_tail = 1u;
      s_ovf = 0u;
      s_stop = kUnseen;
      s_m = 0ull;
      s_a = 0ull;
    }
    __syncthreads();

    // forward: level by level, a thread per frontier vertex over its out-arcs;
    // the first to reach w claims it for level+1 and queues it, and every
    // arc into a level+1 vertex adds the tail's (final) count
    uint32_t qb = 0, qe = 1, level = 0;
    uint64_t my_m = 0, my_a = 0;
    bool my_ovf = false;
    while (qb < qe) {
      for (uint32_t q = qb + tid; q < qe; q += BLOCK) {
        const uint32_t v = queue[q];
        const ull sv = sig[v];
        const int64_t e0 = G.rp[v], e1 = G.rp[v + 1];
        my_m += (uint64_t)(e1 - e0);
        for (int64_t e = e0; e < e1; e += 4) {
          // the arc heads of a chunk are loaded before any is used
          uint32_t wq[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) wq[j] = (e + j < e1) ? (uint32_t)G.col[e + j] : kUnseen;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const uint32_t w = wq[j];
            if (w == kUnseen) break;
            uint32_t d = dist[w];
            if (d == kUnseen) {
              const uint32_t old = atomicCAS(&dist[w], kUnseen, level + 1);
              if (old == kUnseen) {
                queue[atomicAdd(&s_tail, 1u)] = (uint16_t)w;
                d = level + 1;
              } else {
                d = old;
              }
            }
            if (d == level + 1) {
              const ull o = atomicAdd(&sig[w], sv);
              if (o + sv < o) my_ovf = true;  // the exact sum passed 2^64 - 1
              ++my_a;
            }
          }
        }
      }
      __syncthreads();  // level+1 complete
      qb = qe;
      qe = s_tail;
      ++level;
      if (tid == 0) lstart[level + 1] = (uint16_t)qe;
      __syncthreads();  // every thread has read the tail before the next appends
    }
    const uint32_t nlev = level;  // levels 0 .. nlev-1 hold vertices
    atomicAdd(&s_m, (unsigned long long)my_m);
    atomicAdd(&s_a, (unsigned long long)my_a);
    if (my_ovf) s_ovf = 1u;
    // shallowest target level: the backward stops there (delta_s(r) depends
    // only on deeper vertices)
    if (A.full) {
      if (tid == 0) s_stop = 0u;
    } else if (A.ntgt > 0) {
      for (uint32_t q = tid; q < qe; q += BLOCK) {
        const uint32_t v = queue[q];
        if (A.tgt_of[v] >= 0) atomicMin(&s_stop, dist[v]);
      }
    }
    __syncthreads();
    if (tid == 0) {
      A.cnt[(size_t)i * 3 + 0] = qe;
      A.cnt[(size_t)i * 3 + 1] = s_m;
      A.cnt[(size_t)i * 3 + 2] = s_a;
      A.ovf[i] = s_ovf;
    }
    const uint32_t stop = s_stop;
    if (A.xdist) {  // exports of the forward state, before psi takes sigma's words
      for (uint32_t v = tid; v < n; v += BLOCK) {
        const uint32_t d = dist[v];
        A.xdist[(size_t)i * n + v] = d == kUnseen ? ~0ull : (uint64_t)d;
        A.xsig[(size_t)i * n + v] = sig[v];
      }
    }
    __syncthreads();

    // backward, deepest level first: psi(v) = 1/sigma(v) + sum of psi(w) over
    // out-arcs (v, w) with w one level deeper, in arc order
    if (stop != kUnseen) {
      for (int lv = (int)nlev - 1; lv >= (int)stop; --lv) {
        const uint32_t b0 = lstart[lv], b1 = lstart[lv + 1];
        for (uint32_t q = b0 + tid; q < b1; q += BLOCK) {
          const uint32_t v = queue[q];
          double acc = 0.0;
          const int64_t e0 = G.rp[v], e1 = G.rp[v + 1];
          for (int64_t e = e0; e < e1; e += 4) {
            uint32_t wq[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) wq[j] = (e + j < e1) ? (uint32_t)G.col[e + j] : kUnseen;
#pragma unroll
            for (int j = 0; j < 4; ++j)  // arc order
              if (wq[j] != kUnseen && dist[wq[j]] == (uint32_t)lv + 1u) acc += __longlong_as_double((long long)sig[wq[j]]);
          }
          const double sv = (double)sig[v];
          sig[v] = (ull)__double_as_longlong(acc + 1.0 / sv);  // psi(v)
          const double dl = sv * acc;
          if (A.xdel) A.xdel[(size_t)i * n + v] = dl;
          if (A.ntgt > 0) {
            const int32_t t = A.tgt_of[v];
            if (t >= 0) A.res[(size_t)i * A.ntgt + t] = (lv > 0) ? dl : 0.0;
          }
        }
        __syncthreads();
      }
    }
    __syncthreads();  // the next source overwrites the LDS state
  }
}

// Reachability of Def.3 from `root` (on the transpose for RV(r), on the graph
// for the forward reach of r) in one workgroup: visited bits and the BFS
// queue live in LDS, levels are separated by barriers, and the visited
// bitmap is written out at the end.  For n < 2^16.
constexpr int kReachBlock = 1024;

size_t lds_reach_bytes(int64_t n) { return (size_t)4 * (((size_t)n + 31) / 32) + (size_t)2 * (size_t)n + 64; }

__global__ __launch_bounds__(kReachBlock) void k_lds_reach(const int64_t *rp, const int32_t *col, int32_t n,
                                                          int32_t root, uint32_t *bitmap_out) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t words = ((uint32_t)n + 31) / 32;
  uint32_t *vis = reinterpret_cast<uint32_t *>(smem);
  uint16_t *queue = reinterpret_cast<uint16_t *>(smem + 4 * (size_t)words);
  __shared__ uint32_t s_tail;
  const uint32_t tid = threadIdx.x;
  for (uint32_t w = tid; w < words; w += kReachBlock) vis[w] = 0u;
  __syncthreads();
  if (tid == 0) {
    vis[(uint32_t)root >> 5] = 1u << ((uint32_t)root & 31);
    queue[0] = (uint16_t)root;
    s_tail = 1u;
  }
  __syncthreads();
  uint32_t qb = 0, qe = 1;
  while (qb < qe) {
    for (uint32_t q = qb + tid; q < qe; q += kReachBlock) {
      const uint32_t v = queue[q];
      const int64_t e0 = rp[v], e1 = rp[v + 1];
      for (int64_t e = e0; e < e1; e += 4) {
        uint32_t wq[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) wq[j] = (e + j < e1) ? (uint32_t)col[e + j] : kUnseen;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t w = wq[j];
          if (w == kUnseen) break;
          const uint32_t bit = 1u << (w & 31);
          if ((vis[w >> 5] & bit) == 0u && (atomicOr(&vis[w >> 5], bit) & bit) == 0u)
            queue[atomicAdd(&s_tail, 1u)] = (uint16_t)w;
        }
      }
    }
    __syncthreads();
    qb = qe;
    qe = s_tail;
    __syncthreads();
  }
  for (uint32_t w = tid; w < words; w += kReachBlock) bitmap_out[w] = vis[w];
}

bool lds_reach_fits(const Graph *g) { return g->n >= 1 && g->n < 65536 && lds_reach_bytes(g->n) <= g->lds_block_bytes; }

hipError_t launch_lds_reach(const Graph *g, const int64_t *rp, const int32_t *col, int32_t root, uint32_t *bitmap,
                            hipStream_t st) {
  const size_t shm = lds_reach_bytes(g->n);
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(&k_lds_reach), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)shm) != hipSuccess)
    (void)hipGetLastError();
  hipLaunchKernelGGL(k_lds_reach, dim3(1), dim3(kReachBlock), shm, st, rp, col, (int32_t)g->n, root, bitmap);
  return hipGetLastError();
}

// ------------------------------------------------------------------ host

// Device and pinned host scratch of the LDS engine, grown on demand.
static bcd_status lds_scratch(Workspace *ws, size_t dev_bytes, size_t host_bytes) {
  if (dev_bytes > ws->lds_dev_bytes) {
    if (ws->lds_dev) (void)hipFree(ws->lds_dev);
    ws->lds_dev = nullptr;
    ws->lds_dev_bytes = 0;
    if (hipMalloc(&ws->lds_dev, dev_bytes) != hipSuccess) {
      (void)hipGetLastError();
      ws->lds_dev = nullptr;
      return fail(BCD_ERR_OUT_OF_MEMORY, "LDS engine buffers");
    }
    ws->lds_dev_bytes = dev_bytes;
  }
  if (host_bytes > ws->lds_host_bytes) {
    if (ws->lds_host) (void)hipHostFree(ws->lds_host);
    ws->lds_host = nullptr;
    ws->lds_host_bytes = 0;
    if (hipHostMalloc(&ws->lds_host, host_bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      ws->lds_host = nullptr;
      return fail(BCD_ERR_OUT_OF_MEMORY, "LDS engine staging");
    }
    ws->lds_host_bytes = host_bytes;
  }
  return BCD_OK;
}

static size_t align8(size_t x) { return (x + 7) & ~(size_t)7; }

// One launch over `k` sources.  Inputs (sources, then the target map) are
// staged contiguously and go down in one copy; results (dependencies, then
// counters, then overflow flags) come back in one copy.
static bcd_status lds_launch(Graph *g, Workspace *ws, const int32_t *src, int64_t k, const std::vector<int32_t> &tgt,
                             bool full, uint64_t *xdist, unsigned long long *xsig, double *xdel, double *dep,
                             uint64_t *cnt, uint32_t *ovf, float *ms) {
  if (k > INT32_MAX) return fail(BCD_ERR_INVALID_ARG, "too many sources for one launch");
  const size_t n = (size_t)g->n;
  const int ntgt = (int)tgt.size();
  const size_t in_src = align8((size_t)k * 4), in_tgt = ntgt > 0 ? align8(n * 4) : 0;
  const size_t out_res = (size_t)k * (size_t)ntgt * 8, out_cnt = (size_t)k * 24, out_ovf = align8((size_t)k * 4);
  const size_t in_bytes = in_src + in_tgt, out_bytes = out_res + out_cnt + out_ovf;
  STCHK(lds_scratch(ws, in_bytes + out_bytes, std::max(in_bytes, out_bytes)));
  unsigned char *hb = reinterpret_cast<unsigned char *>(ws->lds_host);
  unsigned char *db = reinterpret_cast<unsigned char *>(ws->lds_dev);
  std::memcpy(hb, src, (size_t)k * 4);
  if (ntgt > 0) {
    int32_t *to = reinterpret_cast<int32_t *>(hb + in_src);
    std::fill(to, to + n, -1);
    for (int t = 0; t < ntgt; ++t) to[tgt[(size_t)t]] = t;
  }
  hipStream_t st = ws->stream;
  HIPCHK(hipMemcpyAsync(db, hb, in_bytes, hipMemcpyHostToDevice, st));
  LdsArgs A;
  A.src = reinterpret_cast<const int32_t *>(db);
  A.k = (int)k;
  A.tgt_of = ntgt > 0 ? reinterpret_cast<const int32_t *>(db + in_src) : nullptr;
  A.ntgt = ntgt;
  A.full = full ? 1 : 0;
  A.res = reinterpret_cast<double *>(db + in_bytes);
  A.cnt = reinterpret_cast<uint64_t *>(db + in_bytes + out_res);
  A.ovf = reinterpret_cast<uint32_t *>(db + in_bytes + out_res + out_cnt);
  A.xdist = xdist;
  A.xsig = xsig;
  A.xdel = xdel;
  const size_t shm = lds_bytes_for(g->n);
  // allow dynamic LDS up to the size lds_fits checked (a no-op below 64 KiB)
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(&k_lds_pass<kLdsBlock>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm) != hipSuccess)
    (void)hipGetLastError();
  // as many workgroups as fit on the CUs at once (LDS-bound), each taking
  // sources in turn
  const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(8, (int64_t)(g->lds_block_bytes / shm)));
  const int grid = (int)std::min<int64_t>(k, (int64_t)g->cus * per_cu);
  const bool timed = ms != nullptr;
  if (timed) HIPCHK(hipEventRecord(ws->event_pair(0).first, st));
  hipLaunchKernelGGL(k_lds_pass<kLdsBlock>, dim3(grid), dim3(kLdsBlock), shm, st, g->dev(), A);
  HIPCHK(hipGetLastError());
  if (timed) HIPCHK(hipEventRecord(ws->event_pair(0).second, st));
  HIPCHK(hipMemcpyAsync(hb, db + in_bytes, out_bytes, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (timed) HIPCHK(hipEventElapsedTime(ms, ws->event_pair(0).first, ws->event_pair(0).second));
  if (dep && out_res) std::memcpy(dep, hb, out_res);
  std::memcpy(cnt, hb + out_res, out_cnt);
  std::memcpy(ovf, hb + out_res + out_cnt, (size_t)k * 4);
  return BCD_OK;
}

bcd_status run_lds(Graph *g, Workspace *ws, const std::vector<int32_t> &src, const std::vector<int32_t> &tgt,
                   bool want_counters, SourceRun &out) {
  if (!lds_fits(g))
    return fail(BCD_ERR_UNSUPPORTED, "the LDS engine needs an unweighted graph whose per-source state fits one "
                                     "workgroup's LDS (16 bytes per vertex)");
  const size_t ns = src.size();
  const int ntgt = (int)tgt.size();
  out.dep.assign(ns * (size_t)ntgt, 0.0);
  if (want_counters) out.counters.assign(ns * 3, 0);
  out.width = 1;
  out.te = out.reached = out.dag = 0;
  if (ns == 0) return BCD_OK;
  std::vector<uint64_t> cnt(ns * 3);
  std::vector<uint32_t> ovf(ns);
  const bool profiling = g->profiling.load();
  float ms = 0.0f;
  STCHK(lds_launch(g, ws, src.data(), (int64_t)ns, tgt, false, nullptr, nullptr, nullptr, out.dep.data(), cnt.data(),
                   ovf.data(), profiling ? &ms : nullptr));
  uint64_t tot[C_COUNT] = {0};
  bool any_ovf = false;
  for (size_t i = 0; i < ns; ++i) {
    tot[C_FWD_VPAIRS] += cnt[i * 3 + 0];
    tot[C_FWD_APAIRS] += cnt[i * 3 + 1];
    tot[C_FWD_DPAIRS] += cnt[i * 3 + 2];
    any_ovf = any_ovf || ovf[i] != 0u;
  }
  if (want_counters) out.counters = cnt;
  out.te = tot[C_FWD_APAIRS];
  out.reached = tot[C_FWD_VPAIRS];
  out.dag = tot[C_FWD_DPAIRS];
  if (profiling) {
    // one launch does both passes; its bytes are the forward model's
    const double fb = 32.0 * tot[C_FWD_VPAIRS] + 8.0 * tot[C_FWD_APAIRS] + 8.0 * tot[C_FWD_DPAIRS];
    g->add_profile(0, 1, (double)ms, tot + C_FWD_VPAIRS, fb);
  }
  if (any_ovf) return fail(BCD_ERR_SIGMA_OVERFLOW, "a shortest-path count exceeded 2^64 - 1");
  return BCD_OK;
}

bcd_status multi_source_pass_lds(Graph *g, Workspace *ws, const int32_t *sources, int64_t k, uint64_t *dist,
                                 uint64_t *sigma, double *delta) {
  if (!lds_fits(g))
    return fail(BCD_ERR_UNSUPPORTED, "the LDS engine needs an unweighted graph whose per-source state fits one "
                                     "workgroup's LDS (16 bytes per vertex)");
  const size_t kn = (size_t)k * (size_t)g->n;
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
  hipError_t e = hipMemsetAsync(dl, 0, kn * 8, ws->stream);
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "export setup");
  }
  std::vector<uint64_t> cnt((size_t)k * 3);
  std::vector<uint32_t> ovf((size_t)k);
  bcd_status rc = lds_launch(g, ws, sources, k, std::vector<int32_t>{}, true, dd, ds, dl, nullptr, cnt.data(),
                             ovf.data(), nullptr);
  if (rc == BCD_OK) {
    e = hipSuccess;
    if (dist) e = hipMemcpy(dist, dd, kn * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess && sigma) e = hipMemcpy(sigma, ds, kn * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess && delta) e = hipMemcpy(delta, dl, kn * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = hip_fail(e, "export copy");
  }
  cleanup();
  if (rc == BCD_OK)
    for (int64_t i = 0; i < k; ++i)
      if (ovf[(size_t)i]) return fail(BCD_ERR_SIGMA_OVERFLOW, "a shortest-path count exceeded 2^64 - 1");
  return rc;
}

}  // namespace bcd
