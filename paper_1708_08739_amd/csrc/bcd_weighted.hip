// Weighted graphs (positive integer arc lengths, Section 2): the per-source
// pass for 64 sources per wavefront lane group.
//
//   1. distances: rounds of label-correcting relaxation; lane b lowers
//      dist_b(w) with atomicMin and flags (g, w) for the next round;
//   2. shortest-path-DAG in-degrees: for every reached (g, w), count the
//      in-arcs (u, w) with dist_b(u) + len(u, w) = dist_b(w) (a pull over the
//      reverse graph, no atomics), and store each in-arc's lanes of that test
//      as one 64-bit mask per (group, arc), so that steps 3 and 4 find the
//      DAG lanes of an arc in one word instead of a distance per lane;
//   3. path counts in topological rounds: a lane of a vertex is ready when
//      all its DAG in-arcs have pushed; it then pushes sigma along its DAG
//      out-arcs and counts them down (Kahn's order on each source's SPD);
//   4. backward: Eq.(4) over the rounds of step 3 in reverse -- every DAG
//      successor of v became ready in a later round, so its psi is final.
// Step 3's round of a vertex plays the role of the BFS level of the
// unweighted engine; the backward computes psi only on lanes where the
// vertex is a target or lies below one (marks OR'd along the sigma pushes).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/bcd.h"
#include "bcd_device.h"
#include "bcd_host_internal.h"

namespace bcd {

constexpr uint32_t kInf = 0xFFFFFFFFu;

__global__ void k_w_init(BatchState S, const uint32_t *items0, const ull *masks0, const uint32_t *dest0, int k) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    const uint32_t it = items0[i];
    const ull m = masks0[i];
    S.fr[it] = m;       // topological round 0
    S.items[dest0[i]] = it;
    S.chg[it] = m;      // relaxation round 0: the sources changed
    S.bq[i] = it;
    S.rl[i] = it;
    S.vis[it] = m;      // reached lanes
    for (int b = 0; b < kLanes; ++b)
      if ((m >> b) & 1ull) {
        S.sig[(size_t)it * kLanes + b] = 1ull;
        S.wd[(size_t)it * kLanes + b] = 0u;
      }
  }
  if (blockIdx.x == 0 && threadIdx.x < (unsigned)S.P) S.off[threadIdx.x] = (uint64_t)threadIdx.x * S.capP;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    S.bqn[0] = (uint32_t)k;
    S.bqn[1] = 0u;
    S.bqn[2] = 0u;
    *S.rln = (uint32_t)k;
  }
}

// Lane compaction for one work item: the A lanes of `em` are renumbered
// 0..A-1 in lane order; lane L of the wavefront then serves source lane
// `src` (the one of number L mod A) on arc slot L / A of `slots` = 64 / A
// (slot >= slots: idle).  With few lanes per item the wavefront thus covers
// `slots` arcs of every source at once instead of one.  Wave-uniform `em`.
struct Compact {
  int A, slots, j, slot, src;
};
// Arcs per slot per step of the relaxation: four, so that each lane has four
// distance reads in flight before it waits (a full-width R-MAT 18 batch of
// 8,192 sources: 0.94-0.97 s with one, 0.90-0.92 with two, 0.855-0.88 with
// four, 0.846-0.854 with eight, which needs 74 VGPRs instead of 64).
constexpr int kWU = 4;

// Orders this wavefront's LDS accesses before and after the call (lanes of
// one wavefront exchanging values through LDS).
static __device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// 64-bit lane shuffle (any source lane, every lane taking part).
static __device__ __forceinline__ ull shfl64_w(ull x, int src) {
  const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)x, src);
  const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(x >> 32), src);
  return ((ull)hi << 32) | lo;
}

static __device__ __forceinline__ Compact compact_lanes(ull em, bool mine) {
  Compact c;
  const int lane = lane_id();
  c.A = __popcll(em);
  c.slots = kLanes / c.A;
  // lane of number r learns its lane id (push: a bijection of all 64 lanes)
  const int rk = mine ? lanes_below(em) : c.A + lanes_below(~em);
  const int id = __builtin_amdgcn_ds_permute(rk * 4, lane);
  c.j = lane % c.A;
  c.slot = lane / c.A;
  c.src = __shfl(id, c.j);
  return c;
}

// One relaxation round.  Input: queue bq[round&1] (length bqn[round%3]) with
// changed-lane masks chg[round&1]; output: bq[(round+1)&1], chg[(round+1)&1],
// length bqn[(round+1)%3]; bqn[(round+2)%3] is zeroed for the round after.
// Lanes are compacted per item (compact_lanes).
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_w_relax(DevGraph G, BatchState S, int round) {
  const uint64_t n = (uint64_t)S.n;
  const uint64_t GN = (uint64_t)S.G * n;
  const uint32_t count = S.bqn[round % 3];
  if (blockIdx.x == 0 && threadIdx.x == 0) S.bqn[(round + 2) % 3] = 0u;
  const uint32_t *qin = S.bq + (uint64_t)(round & 1) * GN;
  uint32_t *qout = S.bq + (uint64_t)((round + 1) & 1) * GN;
  uint32_t *qout_n = &S.bqn[(round + 1) % 3];
  ull *ccur = S.chg + (uint64_t)(round & 1) * GN;
  ull *cnxt = S.chg + (uint64_t)((round + 1) & 1) * GN;
  const int lane = lane_id();
  uint64_t c_r = 0;
  const uint64_t wave = ((uint64_t)blockIdx.x * BLOCK + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * BLOCK) >> 6;
  constexpr int kCap = 128;
  __shared__ uint32_t qst_all[(BLOCK / 64) * kCap];
  __shared__ uint32_t rst_all[(BLOCK / 64) * kCap];
  uint32_t *qst = qst_all + (threadIdx.x >> 6) * kCap;
  uint32_t *rst = rst_all + (threadIdx.x >> 6) * kCap;
  // per slot: the lanes that improved the slot's head in this step, and those
  // that reached it first, combined so that the head's flags take one atomic
  // per step, not one per source
  __shared__ ull cm_all[BLOCK], cr_all[BLOCK];
  ull *cm = cm_all + (threadIdx.x & ~63u);
  ull *cr = cr_all + (threadIdx.x & ~63u);
  cm[lane] = 0ull;
  cr[lane] = 0ull;
  wave_lds_sync();
  int nq = 0, nr = 0;
  for (uint64_t i = wave; i < count; i += nwaves) {
    const uint32_t it = qin[i];
    const uint32_t g = (uint32_t)(it / n);
    const uint32_t v = (uint32_t)(it - (uint64_t)g * n);
    const uint64_t gbase = (uint64_t)g * n;
    const ull mask = ccur[it];
    if (lane == 0) ccur[it] = 0ull;  // the owner retires its flag; others write cnxt only
    if (mask == 0ull) continue;
    const Compact cp = compact_lanes(mask, (mask >> lane) & 1ull);
    const bool on = cp.slot < cp.slots;
    const uint32_t dv = on ? S.wd[(uint64_t)it * kLanes + (uint32_t)cp.src] : kInf;
    const bool live = on && dv != kInf;
    const ull bit = 1ull << cp.src;
    const int64_t e0 = G.rp[v], e1 = G.rp[v + 1];
    if (lane == 0) c_r += (uint64_t)cp.A * (uint64_t)(e1 - e0);
    const int64_t stepw = (int64_t)cp.slots * kWU;
    for (int64_t e = e0; e < e1; e += stepw) {
      uint32_t wq[kWU], nd[kWU], dw[kWU];
#pragma unroll
      for (int u = 0; u < kWU; ++u) {
        const int64_t ea = e + (int64_t)u * cp.slots + cp.slot;
        wq[u] = 0u;
        nd[u] = kInf;
        if (live && ea < e1) {
          const uint2 a = G.arcw[ea];
          wq[u] = a.x;
          nd[u] = dv + a.y;
        }
      }
#pragma unroll
      for (int u = 0; u < kWU; ++u) dw[u] = nd[u] != kInf ? S.wd[(gbase + wq[u]) * kLanes + (uint32_t)cp.src] : 0u;
      // a lower tentative distance: lower it (the minimum wins whatever the
      // order) and flag the vertex for the next round; a flag raised by a
      // value another wavefront has already beaten only costs a re-scan
      bool imp[kWU];
#pragma unroll
      for (int u = 0; u < kWU; ++u) {
        imp[u] = nd[u] != kInf && nd[u] < dw[u];
        if (imp[u])
          __hip_atomic_fetch_min(&S.wd[(gbase + wq[u]) * kLanes + (uint32_t)cp.src], nd[u], __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
      }
#pragma unroll
      for (int u = 0; u < kWU; ++u) {
        if (__ballot(imp[u]) == 0ull) continue;  // nothing improved in this step (wave-uniform)
        // a lane that read the head unreached: the wavefront whose lowering
        // of a lane lands first read it unreached, so the pair's first reach
        // is among these and the reached list needs no atomic for the others
        const bool fst = imp[u] && dw[u] == kInf;
        if (imp[u]) __hip_atomic_fetch_or(&cm[cp.slot], bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        if (fst) __hip_atomic_fetch_or(&cr[cp.slot], bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        wave_lds_sync();
        ull m = 0ull, mr = 0ull;
        if (cp.j == 0 && on) {
          m = cm[cp.slot];
          mr = cr[cp.slot];
          cm[cp.slot] = 0ull;
          cr[cp.slot] = 0ull;
        }
        wave_lds_sync();
        bool fq = false, fr = false;
        if (m != 0ull) fq = atomicOr(&cnxt[gbase + wq[u]], m) == 0ull;
        if (mr != 0ull) fr = atomicOr(&S.vis[gbase + wq[u]], mr) == 0ull;
        stage_lanes<kCap>(qst, nq, fq, (uint32_t)(gbase + wq[u]), qout_n, qout, 0, GN, nullptr);
        stage_lanes<kCap>(rst, nr, fr, (uint32_t)(gbase + wq[u]), S.rln, S.rl, 0, GN, nullptr);
      }
    }
  }
  stage_flush(qst, nq, qout_n, qout, 0, GN, nullptr);
  stage_flush(rst, nr, S.rln, S.rl, 0, GN, nullptr);
  flush_counters<BLOCK>(S.ctr, S.ctr_slots, C_RLX_APAIRS, c_r, 0, 0, false, S.flags);
}

// DAG in-degree of every reached (g, w) on each lane, pulled over in-arcs.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_w_count(DevGraph G, BatchState S) {
  const uint64_t n = (uint64_t)S.n;
  const uint64_t GN = (uint64_t)S.G * n;
  uint32_t count = *S.rln;
  if (count > GN) count = (uint32_t)GN;
  const int lane = lane_id();
  uint64_t c_v = 0, c_a = 0, c_d = 0;
  const uint64_t wave = ((uint64_t)blockIdx.x * BLOCK + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * BLOCK) >> 6;
  for (uint64_t i = wave; i < count; i += nwaves) {
    const uint32_t it = S.rl[i];
    const uint32_t g = (uint32_t)(it / n);
    const uint32_t w = (uint32_t)(it - (uint64_t)g * n);
    const uint64_t gbase = (uint64_t)g * n;
    const uint32_t dw = S.wd[(uint64_t)it * kLanes + lane];
    const bool fin = dw != kInf;
    uint32_t c = 0;
    const int64_t e0 = G.irp[w], e1 = G.irp[w + 1];
    ull *dm = S.dagm + (uint64_t)g * (uint64_t)G.m;
    for (int64_t e = e0; e < e1; e += 8) {
      const int cc = (int)((e1 - e) < 8 ? (e1 - e) : 8);
      uint32_t du[8], ln[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        du[q] = kInf;
        ln[q] = 0u;
        if (q < cc && fin) {
          const uint2 a = G.iarc[e + q];
          ln[q] = a.y;
          du[q] = S.wd[(gbase + a.x) * kLanes + lane];
        }
      }
      // lane q keeps the DAG lanes of in-arc e + q; the eight masks go out as
      // one 64-byte store
      ull mine = 0ull;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const bool dag = du[q] != kInf && du[q] + ln[q] == dw;
        if (dag) ++c;
        const ull bq = __ballot(dag);
        if (lane == q) mine = bq;
      }
      if (lane < cc) dm[e + lane] = mine;
    }
    S.wc[(uint64_t)it * kLanes + lane] = c;
    const ull fm = __ballot(fin);
    c_d += c;
    if (lane == 0) {
      c_v += (uint64_t)__popcll(fm);
      c_a += (uint64_t)__popcll(fm) * (uint64_t)(G.rp[w + 1] - G.rp[w]);
    }
  }
  flush_counters<BLOCK>(S.ctr, S.ctr_slots, C_FWD_VPAIRS, c_v, c_a, c_d, false, S.flags);
}

// One topological round: items whose lanes became ready push sigma along
// their DAG out-arcs; a lane of w whose last DAG in-arc pushed is ready next
// round.  Level lists, rotation of the mask arrays and target bookkeeping
// mirror the unweighted forward kernel.  A wavefront lane takes one out-arc
// of the item and reads the arc's DAG mask word, so the DAG test costs one
// load per arc for all 64 sources; pushes happen only on the (source, arc)
// pairs of the DAG, and a head's ready and below-target lanes take one atomic
// each.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_w_sigma(DevGraph G, BatchState S, int level) {
  const uint64_t n = (uint64_t)S.n;
  const uint64_t GN = (uint64_t)S.G * n;
  const int P = S.P;
  const PartView pv = part_view<BLOCK>(P);
  const uint64_t base = S.off[(uint64_t)level * P + pv.p];
  const uint64_t count = S.cnt[(uint64_t)level * P + pv.p];
  const uint64_t nbase = base + count;
  const uint64_t rend = (uint64_t)(pv.p + 1) * S.capP;
  if (pv.thread == 0) S.off[(uint64_t)(level + 1) * P + pv.p] = nbase;
  if (nbase > rend) return;  // capacity exceeded earlier (workgroup-uniform test): batch is redone
  const int lane = lane_id();
  ull *cur = S.fr + (uint64_t)(level % 3) * GN;
  ull *nxt = S.fr + (uint64_t)((level + 1) % 3) * GN;
  ull *old = S.fr + (uint64_t)((level + 2) % 3) * GN;
  if (level > 0) {
    const uint64_t pb = S.off[(uint64_t)(level - 1) * P + pv.p];
    const uint64_t pc = S.cnt[(uint64_t)(level - 1) * P + pv.p];
    for (uint64_t i = pv.thread; i < pc; i += pv.nthreads) old[S.items[pb + i]] = 0ull;
  }
  bool ovf = false;
  const uint64_t wave = pv.wave;
  const uint64_t nwaves = pv.nwaves;
  uint32_t *next_cnt = &S.cnt[(uint64_t)(level + 1) * P + pv.p];
  constexpr int kCap = 256;
  __shared__ uint32_t st_all[(BLOCK / 64) * kCap];
  uint32_t *stg = st_all + (threadIdx.x >> 6) * kCap;
  int nst = 0;
  for (uint64_t i = wave; i < count; i += nwaves) {
    const uint32_t it = S.items[base + i];
    const uint32_t g = (uint32_t)(it / n);
    const uint32_t v = (uint32_t)(it - (uint64_t)g * n);
    const uint64_t gbase = (uint64_t)g * n;
    const ull mask = cur[it];
    if (lane == 0) S.imask[base + i] = mask;
    const bool is_tgt = S.tgt_of[v] >= 0;
    if (is_tgt && lane == 0) atomicMin(S.tmin, (uint32_t)level);
    if (mask == 0ull) continue;
    // lanes on which v is a target or lies below one: final now (every DAG
    // in-arc of a ready lane has pushed); the backward reads only these
    // (an atomic: waves pushing to v's other, not yet ready lanes may add
    // their bits in this round)
    ull dnv = S.wdn[it];
    if (is_tgt) {
      dnv |= mask;
      if (lane == 0) atomicOr(&S.wdn[it], mask);
    }
    const ull *dm = S.dagm + (uint64_t)g * (uint64_t)G.m;
    const uint64_t vrow = (uint64_t)it * kLanes;
    // lane b holds sigma_b(v) of the ready lanes (a per-pair read of the row
    // instead measured 5 % slower on a full-width R-MAT 18 batch)
    const ull svl = ((mask >> lane) & 1ull) ? S.sig[vrow + lane] : 0ull;
    const int64_t e0 = G.rp[v], e1 = G.rp[v + 1];
    // lane j takes arc e + j; its DAG lanes among the ready ones come from
    // the arc's mask word, and only those (source, arc) pairs push
    for (int64_t e = e0; e < e1; e += kLanes) {
      const int64_t ea = e + lane;
      uint32_t x = 0u;
      ull d = 0ull;
      if (ea < e1) {
        const uint2 a = G.arcp[ea];
        x = a.x;
        d = dm[a.y] & mask;
      }
      const uint64_t xrow = (gbase + x) * kLanes;
      ull rdy = 0ull, mdn = 0ull;
      // one source of each arc per pass, lowest first; the passes are few
      // (DAG lanes are a small share of an item's lanes)
      while (__ballot(d != 0ull) != 0ull) {
        const int b = d != 0ull ? __builtin_ctzll(d) : 0;
        const ull sb = shfl64_w(svl, b);  // every lane takes part in the shuffle
        if (d != 0ull) {
          d &= d - 1ull;
          const ull bit = 1ull << b;
          const ull so = atomicAdd(&S.sig[xrow + (uint32_t)b], sb);
          const uint32_t co = atomicSub(&S.wc[xrow + (uint32_t)b], 1u);
          if (so + sb < so) {
            ovf = true;
            atomicOr(&S.ovl[g], bit);
          }
          // the push that completes the head's DAG in-arcs makes the lane ready
          if (co == 1u) rdy |= bit;
          if ((dnv >> b) & 1ull) mdn |= bit;
        }
      }
      if (mdn != 0ull) atomicOr(&S.wdn[gbase + x], mdn);
      bool first = false;
      if (rdy != 0ull) first = atomicOr(&nxt[gbase + x], rdy) == 0ull;
      // the first mark of the head appends it to the next round
      stage_lanes<kCap>(stg, nst, first, (uint32_t)(gbase + x), next_cnt, S.items, nbase, rend, &S.flags[1]);
    }
  }
  stage_flush(stg, nst, next_cnt, S.items, nbase, rend, &S.flags[1]);
  flush_counters<BLOCK>(S.ctr, S.ctr_slots, C_SCRATCH, 0, 0, 0, ovf, S.flags);
}

// Backward over topological round `level`: psi(v) = 1/sigma(v) + sum of
// psi(w) over DAG out-arcs (v, w) of the lane; lanes pruned as in the
// unweighted kernel.  A wavefront lane takes one out-arc and its DAG mask
// word, psi is read only on the DAG (source, arc) pairs, and every source's
// sum runs in arc order, so the result does not depend on the item's lanes.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_w_bwd(DevGraph G, BatchState S, int level, int ntgt, int full) {
  const uint64_t n = (uint64_t)S.n;
  const int P = S.P;
  const PartView pv = part_view<BLOCK>(P);
  const uint64_t base = S.off[(uint64_t)level * P + pv.p];
  const uint64_t count = S.cnt[(uint64_t)level * P + pv.p];
  if (base + count > (uint64_t)(pv.p + 1) * S.capP) return;
  const int lane = lane_id();
  uint64_t c_v = 0, c_a = 0, c_d = 0;
  const uint64_t wave = pv.wave;
  const uint64_t nwaves = pv.nwaves;
  for (uint64_t i = wave; i < count; i += nwaves) {
    const uint32_t it = S.items[base + i];
    const uint32_t g = (uint32_t)(it / n);
    const uint32_t v = (uint32_t)(it - (uint64_t)g * n);
    const uint64_t gbase = (uint64_t)g * n;
    const ull mask = S.imask[base + i];
    const int32_t tg = S.tgt_of[v];
    // a target's dependency reads psi only on lanes where v is a target or
    // lies below one
    const ull dnv = S.wdn[it];
    const bool need = ((mask >> lane) & 1ull) && (full || ((dnv >> lane) & 1ull) || tg >= 0);
    const ull em = __ballot(need);
    if (em == 0ull) continue;
    const ull *dm = S.dagm + (uint64_t)g * (uint64_t)G.m;
    const int64_t e0 = G.rp[v], e1 = G.rp[v + 1];
    double acc = 0.0;  // lane b: the sum of source b, over its DAG arcs in arc order
    uint64_t pairs = 0;
    for (int64_t e = e0; e < e1; e += kLanes) {
      // lane j takes arc e + j and its DAG lanes among the needed ones
      const int64_t ea = e + lane;
      uint32_t x = 0u;
      ull d = 0ull;
      if (ea < e1) {
        const uint2 a = G.arcp[ea];
        x = a.x;
        d = dm[a.y] & em;
      }
      const uint64_t xrow = (gbase + x) * kLanes;
      // eight sources at a time: the lanes of each source's DAG arcs load its
      // psi (all eight loads in flight together), then the source's sum takes
      // them in arc order, so every sum runs in the same order whatever the
      // lanes and batch
      ull rem = em;
      while (rem != 0ull) {
        int bq[8];
        ull aq[8];
        double y[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const bool live = rem != 0ull;
          bq[q] = live ? __builtin_ctzll(rem) : 0;
          aq[q] = __ballot(live && ((d >> bq[q]) & 1ull));
          if (live) rem &= rem - 1ull;
          y[q] = ((aq[q] >> lane) & 1ull) ? S.psi[xrow + (uint32_t)bq[q]] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          ull t = aq[q];
          if (t == 0ull) continue;
          pairs += (uint64_t)__popcll(t);
          double a = __longlong_as_double((long long)read_lane64((ull)__double_as_longlong(acc), bq[q]));
          while (t != 0ull) {
            const int j = __builtin_ctzll(t);
            t &= t - 1ull;
            a += __longlong_as_double((long long)read_lane64((ull)__double_as_longlong(y[q]), j));
          }
          if (lane == bq[q]) acc = a;
        }
      }
    }
    if ((em >> lane) & 1ull) {
      const uint64_t row = (uint64_t)it * kLanes + (uint32_t)lane;
      const double s = (double)S.sig[row];
      const double dl = s * acc;
      S.psi[row] = acc + 1.0 / s;
      if (S.dout) S.dout[row] = dl;
      if (tg >= 0 && tg < ntgt) S.res[((uint64_t)tg * S.G + g) * kLanes + (uint32_t)lane] = (level > 0) ? dl : 0.0;
    }
    if (lane == 0) {
      c_v += (uint64_t)__popcll(em);
      c_a += (uint64_t)__popcll(em) * (uint64_t)(e1 - e0);
      c_d += pairs;
    }
  }
  flush_counters<BLOCK>(S.ctr, S.ctr_slots, C_BWD_VPAIRS, c_v, c_a, c_d, false, S.flags);
}

__global__ void k_w_cleanup(BatchState S) {
  const uint64_t GN = (uint64_t)S.G * (uint64_t)S.n;
  uint64_t count = *S.rln;
  if (count > GN) count = GN;
  const int lane = lane_id();
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t i = wave; i < count; i += nwaves) {
    const uint32_t it = S.rl[i];
    const uint64_t row = (uint64_t)it * kLanes + lane;
    S.wd[row] = kInf;
    S.wc[row] = 0u;
    S.sig[row] = 0ull;
    if (lane == 0) S.vis[it] = 0ull;
    if (lane == 5) S.wdn[it] = 0ull;
    if (lane < 3) S.fr[(uint64_t)lane * GN + it] = 0ull;
    if (lane >= 3 && lane < 5) S.chg[(uint64_t)(lane - 3) * GN + it] = 0ull;
  }
}

__global__ void k_w_export(BatchState S, const int32_t *lane_slot, uint64_t *dist, ull *sigma, double *delta,
                           int64_t k) {
  const uint64_t n = (uint64_t)S.n;
  const uint64_t GN = (uint64_t)S.G * n;
  uint64_t count = *S.rln;
  if (count > GN) count = GN;
  const int lane = lane_id();
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t i = wave; i < count; i += nwaves) {
    const uint32_t it = S.rl[i];
    const uint32_t g = (uint32_t)(it / n);
    const uint32_t v = (uint32_t)(it - (uint64_t)g * n);
    const uint64_t row = (uint64_t)it * kLanes + lane;
    const uint32_t d = S.wd[row];
    if (d == kInf) continue;
    const int32_t slot = lane_slot[g * kLanes + lane];
    if (slot < 0 || slot >= k) continue;
    const uint64_t o = (uint64_t)slot * n + v;
    dist[o] = d;
    sigma[o] = S.sig[row];
    if (delta && S.dout) delta[o] = S.dout[row];
  }
}

#define DISPATCH_BLOCK(L, KERNEL, ...)                                                                  \
  do {                                                                                                  \
    switch ((L).block) {                                                                                \
      case 64: hipLaunchKernelGGL(KERNEL<64>, dim3((L).grid), dim3(64), 0, st, __VA_ARGS__); break;    \
      case 128: hipLaunchKernelGGL(KERNEL<128>, dim3((L).grid), dim3(128), 0, st, __VA_ARGS__); break; \
      case 512: hipLaunchKernelGGL(KERNEL<512>, dim3((L).grid), dim3(512), 0, st, __VA_ARGS__); break; \
      default: hipLaunchKernelGGL(KERNEL<256>, dim3((L).grid), dim3(256), 0, st, __VA_ARGS__); break;  \
    }                                                                                                   \
  } while (0)

hipError_t launch_w_init(const BatchState &S, const uint32_t *items0, const ull *masks0, const uint32_t *dest0, int k,
                         hipStream_t st) {
  const int grid = std::max(1, (k + 255) / 256);
  hipLaunchKernelGGL(k_w_init, dim3(grid), dim3(256), 0, st, S, items0, masks0, dest0, k);
  return hipGetLastError();
}

hipError_t launch_w_relax(const DevGraph &G, const BatchState &S, int round, Launch L, hipStream_t st) {
  DISPATCH_BLOCK(L, k_w_relax, G, S, round);
  return hipGetLastError();
}

hipError_t launch_w_count(const DevGraph &G, const BatchState &S, Launch L, hipStream_t st) {
  DISPATCH_BLOCK(L, k_w_count, G, S);
  return hipGetLastError();
}

hipError_t launch_w_sigma(const DevGraph &G, const BatchState &S, int round, Launch L, hipStream_t st) {
  DISPATCH_BLOCK(L, k_w_sigma, G, S, round);
  return hipGetLastError();
}

hipError_t launch_w_bwd(const DevGraph &G, const BatchState &S, int round, int ntgt, int full, Launch L,
                        hipStream_t st) {
  DISPATCH_BLOCK(L, k_w_bwd, G, S, round, ntgt, full);
  return hipGetLastError();
}

hipError_t launch_w_cleanup(const BatchState &S, Launch L, hipStream_t st) {
  hipLaunchKernelGGL(k_w_cleanup, dim3(L.grid), dim3(256), 0, st, S);
  return hipGetLastError();
}

hipError_t launch_w_export(const BatchState &S, const int32_t *lane_slot, uint64_t *dist, ull *sigma,
                           double *delta, int64_t k, Launch L, hipStream_t st) {
  hipLaunchKernelGGL(k_w_export, dim3(L.grid), dim3(256), 0, st, S, lane_slot, dist, sigma, delta, k);
  return hipGetLastError();
}

}  // namespace bcd

// ================================================================= host

namespace bcd {


template <class T>
static bcd_status walloc(T **p, size_t count) {
  *p = nullptr;
  if (hipMalloc((void **)p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(BCD_ERR_OUT_OF_MEMORY, "device allocation for the weighted engine failed");
  }
  return BCD_OK;
}

bcd_status Workspace::ensure_weighted() {
  if (weighted_ready && weighted_G == G) return BCD_OK;
  release_weighted();
  const size_t GN = (size_t)G * (size_t)n;
  STCHK(walloc(&S.wd, GN * kLanes));
  STCHK(walloc(&S.wc, GN * kLanes));
  STCHK(walloc(&S.chg, 2 * GN));
  STCHK(walloc(&S.bq, 2 * GN));
  STCHK(walloc(&S.bqn, 4));
  STCHK(walloc(&S.rl, GN));
  STCHK(walloc(&S.rln, 1));
  STCHK(walloc(&S.wdn, GN));
  STCHK(walloc(&S.dagm, (size_t)G * (size_t)graph->m));
  HIPCHK(hipMemsetAsync(S.wd, 0xFF, GN * kLanes * sizeof(uint32_t), stream));
  HIPCHK(hipMemsetAsync(S.wdn, 0, GN * sizeof(unsigned long long), stream));
  HIPCHK(hipMemsetAsync(S.wc, 0, GN * kLanes * sizeof(uint32_t), stream));
  HIPCHK(hipMemsetAsync(S.chg, 0, 2 * GN * sizeof(unsigned long long), stream));
  HIPCHK(hipMemsetAsync(S.bqn, 0, 4 * sizeof(uint32_t), stream));
  HIPCHK(hipMemsetAsync(S.rln, 0, sizeof(uint32_t), stream));
  HIPCHK(hipStreamSynchronize(stream));
  weighted_ready = true;
  weighted_G = G;
  return BCD_OK;
}

void Workspace::release_weighted() {
  auto f = [](auto *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
  };
  f(S.wd);
  f(S.wc);
  f(S.chg);
  f(S.bq);
  f(S.bqn);
  f(S.rl);
  f(S.rln);
  f(S.wdn);
  f(S.dagm);
  weighted_ready = false;
}

struct WExport {
  uint64_t *dist = nullptr;
  unsigned long long *sigma = nullptr;
  double *delta = nullptr;
  int64_t k = 0;
};

// One batch of the weighted engine; `k` sources staged in h_items0/h_masks0.
static bcd_status run_one_wbatch(Graph *g, Workspace *ws, int k, int ntgt, bool full, WExport *ex, ProfAcc *prof,
                                 bool *sigma_overflow,
                                 bool copy_res = true, unsigned long long *ovl_out = nullptr) {
  hipStream_t st = ws->stream;
  const DevGraph D = g->dev();
  const bool profiling = g->profiling.load();
  const size_t G64 = (size_t)ws->G * kLanes;
  HIPCHK(hipMemcpyAsync(ws->d_items0, ws->h_items0, (size_t)k * sizeof(uint32_t), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(ws->d_masks0, ws->h_masks0, (size_t)k * sizeof(unsigned long long), hipMemcpyHostToDevice,
                        st));
  for (int attempt = 0;; ++attempt) {
    ws->S.epoch += 1;
    BatchState S = ws->S;
    if (!ex) S.dout = nullptr;
    S.P = ws->batch_parts(k);  // partitions that hold this batch's groups
    const int P = S.P;
    const Launch L = g->launch_parts(P);
    ws->stage_sources_dest(k);
    HIPCHK(hipMemcpyAsync(ws->d_dest0, ws->h_dest0, (size_t)k * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    uint32_t *hc = ws->h_cnt;
    uint32_t *hc0 = hc + kCntStage;
    uint32_t *hm = reinterpret_cast<uint32_t *>(ws->h_misc);
    for (int p = 0; p < P; ++p) hc0[p] = ws->h_cnt0[p];
    HIPCHK(hipMemcpyAsync(&S.cnt[0], hc0, (size_t)P * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    if (ntgt > 0) HIPCHK(hipMemsetAsync(S.res, 0, (size_t)ntgt * G64 * sizeof(double), st));
    HIPCHK(hipMemsetAsync(S.tmin, 0xFF, sizeof(uint32_t), st));
    HIPCHK(hipMemsetAsync(S.flags, 0, 4 * sizeof(uint32_t), st));
    HIPCHK(hipMemsetAsync(S.ovl, 0, (size_t)ws->G * sizeof(unsigned long long), st));
    HIPCHK(launch_w_init(S, ws->d_items0, ws->d_masks0, ws->d_dest0, k, st));
    size_t ev = 0;
    auto rec0 = [&]() -> hipError_t {
      return profiling ? hipEventRecord(ws->event_pair(ev).first, st) : hipSuccess;
    };
    auto rec1 = [&]() -> hipError_t {
      if (!profiling) return hipSuccess;
      hipError_t e = hipEventRecord(ws->event_pair(ev).second, st);
      ++ev;
      return e;
    };
    // 1. distances
    int round = 0;
    for (;;) {
      const int chunk = 8;
      for (int i = 0; i < chunk; ++i, ++round) {
        HIPCHK(rec0());
        HIPCHK(launch_w_relax(D, S, round, L, st));
        HIPCHK(rec1());
      }
      HIPCHK(hipMemcpyAsync(hm, &S.bqn[round % 3], sizeof(uint32_t), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (hm[0] == 0) break;
      if (round > g->n + 16) return fail(BCD_ERR_DEVICE, "relaxation rounds did not converge");
    }
    // 2. DAG in-degrees
    HIPCHK(rec0());
    HIPCHK(launch_w_count(D, S, L, st));
    HIPCHK(rec1());
    // 3. path counts in topological rounds
    std::vector<uint32_t> cntp(hc0, hc0 + P);
    int lmax = -1, level = 0;
    int chunk = std::min(kLevelChunkMax, std::max(4, ws->last_depth + 2));
    uint32_t flags_h[2] = {0, 0}, tmin_h = 0xFFFFFFFFu;
    while (lmax < 0) {
      const int first = level;
      int launched = 0;
      for (; launched < chunk && level <= g->n; ++launched, ++level) {
        HIPCHK(rec0());
        HIPCHK(launch_w_sigma(D, S, level, L, st));
        HIPCHK(rec1());
      }
      HIPCHK(hipMemcpyAsync(hc, &S.cnt[(size_t)(first + 1) * P], (size_t)launched * P * sizeof(uint32_t),
                            hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(hm, S.flags, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(hm + 2, S.tmin, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      flags_h[0] = hm[0];
      flags_h[1] = hm[1];
      tmin_h = hm[2];
      if (flags_h[1]) break;
      for (int i = 0; i < launched; ++i) {
        uint64_t tot = 0;
        for (int p = 0; p < P; ++p) tot += hc[(size_t)i * P + p];
        if (tot == 0) {
          lmax = first + i;
          break;
        }
        cntp.insert(cntp.end(), hc + (size_t)i * P, hc + (size_t)(i + 1) * P);
      }
      if (lmax < 0 && level > g->n) return fail(BCD_ERR_DEVICE, "topological rounds did not terminate");
      chunk = kLevelChunkMax;
    }
    if (flags_h[1]) {
      HIPCHK(launch_w_cleanup(S, L, st));
      STCHK(ws->reset_batch_dense());
      STCHK(ws->grow_items());
      if (attempt > 8) return fail(BCD_ERR_OUT_OF_MEMORY, "frontier item list cannot grow further");
      continue;
    }
    ws->last_depth = lmax;
    if (flags_h[0]) *sigma_overflow = true;
    const size_t fwd_events = ev;
    // 4. backward
    int stop = -1;
    if (full) stop = 0;
    else if (ntgt > 0 && tmin_h != 0xFFFFFFFFu) stop = (int)tmin_h;
    if (stop >= 0)
      for (int lv = lmax; lv >= stop; --lv) {
        HIPCHK(rec0());
        HIPCHK(launch_w_bwd(D, S, lv, ntgt, full ? 1 : 0, L, st));
        HIPCHK(rec1());
      }
    if (ex) HIPCHK(launch_w_export(S, ws->d_lane_slot, ex->dist, ex->sigma, ex->delta, ex->k, L, st));
    if (ntgt > 0 && copy_res)
      HIPCHK(hipMemcpyAsync(ws->h_res, S.res, (size_t)ntgt * G64 * sizeof(double), hipMemcpyDeviceToHost, st));
    if (ovl_out)
      HIPCHK(hipMemcpyAsync(ovl_out, S.ovl, (size_t)ws->G * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    HIPCHK(launch_w_cleanup(S, L, st));
    HIPCHK(launch_ctr_fold(S.ctr, kCtrSlots, S.acc, st));
    HIPCHK(hipMemsetAsync(S.cnt, 0, ((size_t)lmax + 2) * P * sizeof(uint32_t), st));
    HIPCHK(hipStreamSynchronize(st));
    if (profiling && prof) {
      for (size_t i = 0; i < ev; ++i) prof->add(g, i < fwd_events ? 0 : 1, ws->events[i].first, ws->events[i].second);
      // work items: one per (group, vertex, topological round) with ready lanes
      for (size_t l = 0; l * P < cntp.size(); ++l)
        for (int p = 0; p < P; ++p) {
          prof->items[0] += cntp[l * P + p];
          if (stop >= 0 && (int)l >= stop) prof->items[1] += cntp[l * P + p];
        }
    }
    return BCD_OK;
  }
}

static bcd_status wcounters(Workspace *ws, uint64_t *c) { return collect_counters(ws, c, ws->S.acc); }

// Algorithmic bytes per (source, element) pair: 32 per vertex, 12 per arc
// (head index, arc length, head distance), 8 per DAG arc, in each pass.
void record_wprofile(Graph *g, const ProfAcc &p, const uint64_t *c) {
  const double fb = 32.0 * c[C_FWD_VPAIRS] + 12.0 * c[C_FWD_APAIRS] + 8.0 * c[C_FWD_DPAIRS];
  const double bb = 32.0 * c[C_BWD_VPAIRS] + 12.0 * c[C_BWD_APAIRS] + 8.0 * c[C_BWD_DPAIRS];
  g->add_profile(0, p.launches[0], p.ms[0], c + C_FWD_VPAIRS, fb, p.items[0], &p.iv[0], 0, 0.0);
  g->add_profile(1, p.launches[1], p.ms[1], c + C_BWD_VPAIRS, bb, p.items[1], &p.iv[1], 0, 0.0);
}

bcd_status run_staged_wbatch(Graph *g, Workspace *ws, int k, int ntgt, unsigned long long *ovl_out, bool *ovf,
                             ProfAcc *prof) {
  if ((uint64_t)g->n * (uint64_t)g->max_w >= 0xFFFFFFFFull)
    return fail(BCD_ERR_UNSUPPORTED, "n * max weight must stay below 2^32 - 1 for 32-bit distances");
  STCHK(ws->ensure_weighted());
  return run_one_wbatch(g, ws, k, ntgt, false, nullptr, prof, ovf, false, ovl_out);
}

bcd_status run_weighted(Graph *g, Workspace *ws, const std::vector<int32_t> &src, const std::vector<int32_t> &tgt,
                        bool want_counters, SourceRun &out) {
  const bcd_config cfg = g->config();
  if ((uint64_t)g->n * (uint64_t)g->max_w >= 0xFFFFFFFFull)
    return fail(BCD_ERR_UNSUPPORTED, "n * max weight must stay below 2^32 - 1 for 32-bit distances");
  STCHK(ws->ensure_batch(cfg.groups));
  STCHK(ws->ensure_weighted());
  const int ntgt = (int)tgt.size();
  const size_t G64 = (size_t)ws->G * kLanes;
  STCHK(ws->ensure_res((size_t)std::max(ntgt, 1) * G64));
  const size_t ns = src.size();
  out.dep.assign(ns * (size_t)ntgt, 0.0);
  if (want_counters) out.counters.assign(ns * 3, 0);
  // the plain engine on a weighted graph runs one source per batch
  const bool one = want_counters || cfg.engine == BCD_ENGINE_PLAIN;
  const size_t per = one ? 1 : G64;
  out.width = (int32_t)per;
  std::vector<uint32_t> ord;
  STCHK(source_order(g, ws, src, ord));
  ProfAcc prof;
  bool ovf = false;
  uint64_t tot[C_COUNT] = {0};
  // batches b = first, first + stride, ... on workspace w; each source's
  // dependencies go to its own position
  auto stripe = [&](Workspace *w, size_t first, size_t stride, ProfAcc &p, bool &o) -> bcd_status {
    TargetMap tm;
    STCHK(tm.install(w, tgt));
    std::vector<int32_t> bsrc(per);
    for (size_t b0 = first * per; b0 < ns; b0 += stride * per) {
      const int k = (int)std::min(per, ns - b0);
      for (int i = 0; i < k; ++i) bsrc[(size_t)i] = src[ord[b0 + i]];
      w->stage_sources(bsrc.data(), k);
      STCHK(run_one_wbatch(g, w, k, ntgt, false, nullptr, &p, &o));
      for (int i = 0; i < k; ++i)
        for (int t = 0; t < ntgt; ++t) out.dep[(size_t)ord[b0 + i] * ntgt + t] = w->h_res[(size_t)t * G64 + i];
      if (want_counters) {
        uint64_t c[C_COUNT];
        STCHK(wcounters(w, c));
        out.counters[(size_t)ord[b0] * 3 + 0] = c[C_FWD_VPAIRS];
        out.counters[(size_t)ord[b0] * 3 + 1] = c[C_FWD_APAIRS];
        out.counters[(size_t)ord[b0] * 3 + 2] = c[C_FWD_DPAIRS];
        for (int j = 0; j < C_COUNT; ++j) tot[j] += c[j];
      }
    }
    return BCD_OK;
  };
  if (one) {
    STCHK(stripe(ws, 0, 1, prof, ovf));
  } else {
    auto prepare = [&](Workspace *w) -> bcd_status {
      STCHK(w->ensure_batch(cfg.groups));
      STCHK(w->ensure_weighted());
      return w->ensure_res((size_t)std::max(ntgt, 1) * G64);
    };
    STCHK(run_pipelined(g, ws, (ns + per - 1) / per, prepare, stripe, prof, ovf, tot));
    uint64_t t1[C_COUNT];
    STCHK(wcounters(ws, t1));
    for (int j = 0; j < C_COUNT; ++j) tot[j] += t1[j];
  }
  out.te = tot[C_FWD_APAIRS];
  out.reached = tot[C_FWD_VPAIRS];
  out.dag = tot[C_FWD_DPAIRS];
  if (g->profiling.load()) record_wprofile(g, prof, tot);
  if (ovf) return fail(BCD_ERR_SIGMA_OVERFLOW, "a shortest-path count exceeded 2^64 - 1");
  return BCD_OK;
}

bcd_status multi_source_pass_weighted(Graph *g, const int32_t *sources, int64_t k, uint64_t *dist, uint64_t *sigma,
                                      double *delta) {
  const bcd_config cfg = g->config();
  if (k > (int64_t)cfg.groups * kLanes) return fail(BCD_ERR_INVALID_ARG, "k exceeds the batch width");
  if ((uint64_t)g->n * (uint64_t)g->max_w >= 0xFFFFFFFFull)
    return fail(BCD_ERR_UNSUPPORTED, "n * max weight must stay below 2^32 - 1 for 32-bit distances");
  for (int64_t i = 0; i < k; ++i) {
    if (sources[i] < 0 || sources[i] >= g->n) return fail(BCD_ERR_INVALID_ARG, "source out of range");
    for (int64_t j = 0; j < i; ++j)
      if (sources[j] == sources[i] && i / kLanes == j / kLanes) return fail(BCD_ERR_INVALID_ARG, "repeated source");
  }
  Lease ls(g);
  if (!ls.ok()) return fail(BCD_ERR_OUT_OF_MEMORY, "workspace allocation failed");
  STCHK(ls->init_common(g));
  Workspace *ws = ls.w.get();
  STCHK(ws->ensure_batch(cfg.groups));
  STCHK(ws->ensure_weighted());
  STCHK(ws->ensure_dout());
  const size_t G64 = (size_t)ws->G * kLanes;
  const size_t kn = (size_t)k * (size_t)g->n;
  WExport ex;
  ex.k = k;
  STCHK(walloc(&ex.dist, kn));
  bcd_status rc = walloc(&ex.sigma, kn);
  if (rc == BCD_OK) rc = walloc(&ex.delta, kn);
  hipStream_t st = ws->stream;
  std::vector<int32_t> slot(G64, -1);
  for (int64_t i = 0; i < k; ++i) slot[(size_t)i] = (int32_t)i;
  hipError_t e = hipSuccess;
  if (rc == BCD_OK) {
    e = hipMemcpyAsync(ws->d_lane_slot, slot.data(), G64 * sizeof(int32_t), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(ex.dist, 0xFF, kn * 8, st);
    if (e == hipSuccess) e = hipMemsetAsync(ex.sigma, 0, kn * 8, st);
    if (e == hipSuccess) e = hipMemsetAsync(ex.delta, 0, kn * 8, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = hip_fail(e, "export setup");
  }
  bool ovf = false;
  if (rc == BCD_OK) {
    ws->stage_sources(sources, (int)k);
    rc = run_one_wbatch(g, ws, (int)k, 0, true, &ex, nullptr, &ovf);
  }
  if (rc == BCD_OK) {
    e = hipSuccess;
    if (dist) e = hipMemcpy(dist, ex.dist, kn * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess && sigma) e = hipMemcpy(sigma, ex.sigma, kn * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess && delta) e = hipMemcpy(delta, ex.delta, kn * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = hip_fail(e, "export copy");
  }
  if (ex.dist) (void)hipFree(ex.dist);
  if (ex.sigma) (void)hipFree(ex.sigma);
  if (ex.delta) (void)hipFree(ex.delta);
  uint64_t cc[C_COUNT];
  if (rc == BCD_OK) rc = wcounters(ws, cc);
  if (rc == BCD_OK && ovf) rc = fail(BCD_ERR_SIGMA_OVERFLOW, "a shortest-path count exceeded 2^64 - 1");
  return rc;
}

}  // namespace bcd
