// HIP kernels for gfx950 (CDNA4, wave64): the per-source shortest-path pass
// of the paper's Alg.1 / Alg.2 (forward path counting, then the Eq.(4)
// dependency accumulation), the RV(r) reachability traversal of Def.3, and
// a copy probe.
//
// Batched engine layout: a column group is 64 sources, one per wavefront
// lane.  A frontier item is (group g, vertex v) with a 64-bit mask of the
// lanes for which v sits on the current BFS level; lane b works for source b,
// so the 64 path counts of v are one coalesced 512-byte row.  The settled
// lanes and the rotating level masks of (g, v) share one 64-byte record, so
// testing "has source b already settled w" for all 64 sources reads one
// line per arc.  A wavefront takes 1, 2 or 4 items per step (their first
// arcs in separate slots of lanes) to keep several items' loads in flight.
#include <algorithm>

#include "bcd_device.h"

namespace bcd {

// ------------------------------------------------------------ batched

// Level 0: each item is (g, source vertex) with the lanes it is the source
// of; sigma = 1 on those lanes.
__global__ void k_batch_init(BatchState S, const uint32_t *items0, const ull *masks0, const uint32_t *dest0, int k) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    const uint32_t it = items0[i];
    const ull m = masks0[i];
    S.rec[it].fr[0] = m;  // level-0 masks
    S.items[dest0[i]] = it;
    for (int b = 0; b < kLanes; ++b)
      if ((m >> b) & 1ull) S.sig[(size_t)it * kLanes + b] = 1ull;
  }
  // level-0 item-list base of every partition of this batch
  if (blockIdx.x == 0 && threadIdx.x < (unsigned)S.P) S.off[threadIdx.x] = (uint64_t)threadIdx.x * S.capP;
}

// Sum of sigma_b(u) over the in-arcs held by one chunk of lanes whose tail u
// is on the previous level for lane b (pm = lanes of that arc).  The chunk
// holds the arcs of up to K items, 64 / K lanes each (arc lane l belongs to
// the item of slot l / (64 / K), whose group base is in lane l's gbase), and
// an arc adds into its item's accumulator.  With HIT, hit[t] is also set on
// every lane that received a count for item t (the bottom-up kernel's test
// of which lanes reached the level).  Row loads of up to eight
// predecessors are issued before any of them is consumed; the sums are
// exact integers, so the order of the adds does not matter, and an
// unsigned wrap on any add means the true sum exceeds 2^64 - 1.
template <int K, bool HIT = false>
static __device__ __forceinline__ void pull_slots(const BatchState &S, uint64_t gbase, uint32_t u, ull pm, int lane,
                                                  ull (&acc)[K], bool (&lov)[K], bool (&hit)[K], uint64_t &dag_pairs) {
  constexpr int SUB = kLanes / K;
  ull bits = __ballot(pm != 0ull);
  while (bits != 0ull) {
    int j[8];
    int c = 0;
    for (; c < 8 && bits != 0ull; ++c) {
      j[c] = __ffsll((long long)bits) - 1;
      bits &= bits - 1ull;
    }
    // each row load writes its own register, so all eight stay in flight
    ull x[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      x[q] = 0ull;
      if (q < c) {
        const uint32_t uq = read_lane(u, j[q]);
        const ull dq = read_lane64(pm, j[q]);
        const uint64_t gq = read_lane64(gbase, j[q]);
        dag_pairs += (uint64_t)__popcll(dq);  // wave-uniform
        if ((dq >> lane) & 1ull) x[q] = S.sig[(gq + uq) * kLanes + lane];
      }
    }
    if (HIT) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (q < c && ((read_lane64(pm, j[q]) >> lane) & 1ull)) {
          const int slot = j[q] / SUB;
#pragma unroll
          for (int t = 0; t < K; ++t)
            if (slot == t) hit[t] = true;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const ull xq = x[q];
      if (q < c) {
        const int slot = j[q] / SUB;
#pragma unroll
        for (int t = 0; t < K; ++t) {
          if (slot == t) {
            const ull sum = acc[t] + xq;
            if (sum < acc[t]) lov[t] = true;
            acc[t] = sum;
          }
        }
      }
    }
  }
}

// OR of x over the lanes of each item slot (lane l in slot l / (64 / K)),
// into wave-uniform out[]; x must be set on every lane.
template <int K>
static __device__ __forceinline__ void or_slots(ull x, ull (&out)[K]) {
  constexpr int SUB = kLanes / K;
  ull b = __ballot(x != 0ull);
  while (b != 0ull) {
    const int j = __ffsll((long long)b) - 1;
    b &= b - 1ull;
    const ull v = read_lane64(x, j);
#pragma unroll
    for (int t = 0; t < K; ++t)
      if (j / SUB == t) out[t] |= v;
  }
}

// Discovered heads are staged in a per-wavefront LDS buffer and copied to
// the next level's list in blocks: one counter atomic per block instead of
// one per out-arc chunk, which keeps the partition's tail counter cold.
constexpr int kStage = 256;

static __device__ __forceinline__ void flush_stage(const BatchState &S, uint32_t *stage, int &nst,
                                                   uint32_t *next_cnt, uint64_t nbase, uint64_t rend) {
  if (nst == 0) return;
  uint32_t p0 = 0;
  if (lane_id() == 0) p0 = atomicAdd(next_cnt, (uint32_t)nst);
  p0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)p0);
  for (int j = lane_id(); j < nst; j += 64) {
    const uint64_t p = nbase + p0 + (uint64_t)j;
    if (p < rend) S.items[p] = stage[j];
    else atomicOr(&S.flags[1], 1u);
  }
  nst = 0;
}

static __device__ __forceinline__ void append_chunk(const BatchState &S, uint32_t *stage, int &nst,
                                                    uint32_t *next_cnt, uint64_t nbase, uint64_t rend,
                                                    uint64_t gbase, uint32_t w, bool enq) {
  const ull eb = __ballot(enq);
  if (eb == 0ull) return;
  const int c = __popcll(eb);
  if (nst + c > kStage) flush_stage(S, stage, nst, next_cnt, nbase, rend);
  if (enq) stage[nst + lanes_below(eb)] = (uint32_t)(gbase + w);
  nst += c;
}

// One BFS level of the batched forward pass (unweighted graphs).  For every
// item (g, v, mask) on `level`:
//   1. sigma pull: sigma_b(v) = sum of sigma_b(u) over in-arcs (u, v) with u
//      on level-1 for lane b (the shortest-path-DAG predecessors of v), an
//      exact uint64 sum with a carry check on every add; no atomics;
//   2. discovery: for every out-arc (v, w), lanes b in mask for which w is
//      not settled on a level <= `level` are DAG arcs; they are flagged on
//      (g, w) for level+1 with one atomicOr per arc, lanes over arcs, and
//      the first flagger appends (g, w) to the next level's item list.
// A wavefront takes K items per step: each item's first 64 / K in-arcs and
// out-arcs sit in its own slot of lanes, so the dependent loads of K items
// (item -> mask and CSR bounds -> arc heads -> head masks -> flags and
// predecessor rows) are in flight together; arcs past the first 64 / K of
// an item are then taken 64 at a time by the whole wavefront.
// Level masks rotate over four words of the (g, v) record: cur (level), nxt
// (level+1, being built), prv (level-1, read by the pull) and old (level-2,
// retired here).  vis lags: the owner of (g, v) ORs cur into vis during this
// launch, so a reader sees vis | cur, which is the same union either way.
// With bottom-up levels enabled, step 1 is skipped when the level was found
// by k_bu_level (which pulled the counts), and step 2 when level+1 will be;
// the item masks are recorded for the backward either way.
// At least 6 waves per SIMD: with the below-target marks, asking for 7
// (72 VGPRs) made the compiler spill 44 bytes per lane and measured 3.5 %
// slower at R-MAT 16 (5 waves: 2 % slower).
template <int BLOCK, int K>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_fwd_level(DevGraph G,
                                                                                                 BatchState S,
                                                                                                 int level) {
  constexpr int SUB = kLanes / K;
  const uint64_t n = (uint64_t)S.n;
  const int P = S.P;
  const PartView pv = part_view<BLOCK>(P);
  const uint64_t base = S.off[(uint64_t)level * P + pv.p];
  const uint64_t count = S.cnt[(uint64_t)level * P + pv.p];
  const uint64_t nbase = base + count;
  const uint64_t rend = (uint64_t)(pv.p + 1) * S.capP;
  if (pv.thread == 0) S.off[(uint64_t)(level + 1) * P + pv.p] = nbase;
  // capacity exceeded (the batch is redone); the test is the same for every
  // thread of the workgroup, so no wave leaves before the counter barrier
  if (nbase > rend) return;
  const int lane = lane_id();
  const int sl = lane % SUB;  // lane within its item slot
  MaskRec *rec = S.rec;
  const int kc = level & 3, kn = (level + 1) & 3, ko = (level + 2) & 3, kp = (level + 3) & 3;

  // retire the masks of level-2 so that word can collect level+2
  if (level >= 2) {
    const uint64_t pb = S.off[(uint64_t)(level - 2) * P + pv.p];
    const uint64_t pc = S.cnt[(uint64_t)(level - 2) * P + pv.p];
    for (uint64_t i = pv.thread; i < pc; i += pv.nthreads) rec[S.items[pb + i]].fr[ko] = 0ull;
  }
  // This launch pulls sigma for the level's items (and settles their lanes)
  // unless the bottom-up kernel already found them with their counts, and
  // discovers level+1 unless that level will be found bottom-up.  Both
  // tests read complete counts, so every workgroup decides alike.
  uint64_t prev = 0;
  if (level >= 1)
    for (int p = 0; p < P; ++p) prev += S.cnt[(uint64_t)(level - 1) * P + p];
  uint64_t cur = 0;
  for (int p = 0; p < P; ++p) cur += S.cnt[(uint64_t)level * P + p];
  const bool pull = !bottom_up_rule(S.bu_den, level, prev, S.gused, S.n);
  const bool disc = !bottom_up_rule(S.bu_den, level + 1, cur, S.gused, S.n);

  // counters, all wave-uniform: (source, vertex), (source, arc) and
  // (source, DAG arc) pairs; items and the out-degree sum over items
  uint64_t c_v = 0, c_a = 0, c_d = 0, c_it = 0, c_ia = 0;
  bool ovf = false;
  const uint64_t step = pv.nwaves * (uint64_t)K;
  uint32_t *next_cnt = &S.cnt[(uint64_t)(level + 1) * P + pv.p];
  __shared__ uint32_t stage_all[(BLOCK / 64) * kStage];
  uint32_t *stage = stage_all + (threadIdx.x >> 6) * kStage;
  int nst = 0;
  uint64_t ii = pv.wave * (uint64_t)K + (uint64_t)(lane / SUB);  // this lane's item
  uint32_t it_next = ii < count ? S.items[base + ii] : 0u;
  for (uint64_t i0 = pv.wave * (uint64_t)K; i0 < count; i0 += step, ii += step) {
    const bool has = ii < count;
    const uint32_t it = it_next;
    if (ii + step < count) it_next = S.items[base + ii + step];  // prefetch the next step's items
    const uint32_t g = (uint32_t)(it / n);
    const uint32_t v = (uint32_t)(it - (uint64_t)g * n);
    const uint64_t gbase = (uint64_t)g * n;
    // independent loads of this slot's item, issued together
    ull mask = 0ull;
    int64_t e0 = 0, e1 = 0, f0 = 0, f1 = 0;
    int32_t tg = -1;
    if (has) {
      mask = rec[it].fr[kc];
      e0 = G.rp[v];
      e1 = G.rp[v + 1];
      if (level > 0 && pull) {
        f0 = G.irp[v];
        f1 = G.irp[v + 1];
      }
      if (pull) tg = S.tgt_of[v];
    }
    const int64_t d1 = disc ? e1 : e0;  // end of the out-arcs to scan
    if (has && sl == 0 && pull) rec[it].vis = rec[it].vis | mask;
    // first chunk of in-arcs (sigma pull) and of out-arcs (discovery) of
    // every slot, interleaved: 1. both index chunks
    const int64_t mi = f0 + sl, mo = e0 + sl;
    uint32_t u = 0, w = 0;
    if (mi < f1) u = (uint32_t)G.icol[mi];
    if (mo < d1) w = (uint32_t)G.col[mo];
    // 2. both mask gathers
    ull pfr = 0ull, svis = 0ull, sfc = 0ull, sfn = 0ull;
    if (mi < f1) pfr = rec[gbase + u].fr[kp];
    if (mo < d1) {
      const MaskRec &R = rec[gbase + w];
      svis = R.vis;
      sfc = R.fr[kc];
      sfn = R.fr[kn];
    }
    const ull pm = pfr & mask;
    // lanes already flagged for level+1 by another wavefront need no atomic
    // (a stale read only costs a redundant atomic)
    const ull dag = (mo < d1) ? (mask & ~(svis | sfc | sfn)) : 0ull;
    // 3. discovery flags, then the predecessor rows; the flag results are
    //    consumed only after the rows
    bool enq = false;
    if (dag != 0ull) enq = (atomicOr(&rec[gbase + w].fr[kn], dag) == 0ull);
    ull acc[K];
    bool lov[K];
#pragma unroll
    for (int t = 0; t < K; ++t) {
      acc[t] = 0ull;
      lov[t] = false;
    }
    // a DAG tail's lanes that are a target or below one: the same record
    // line as its level mask, loaded beside the predecessor rows
    const ull pdn = pm != 0ull ? rec[gbase + u].dn : 0ull;
    pull_slots<K>(S, gbase, u, pm, lane, acc, lov, lov, c_d);
    ull dnacc[K];
#pragma unroll
    for (int t = 0; t < K; ++t) dnacc[t] = 0ull;
    or_slots<K>(pm & pdn, dnacc);
    append_chunk(S, stage, nst, next_cnt, nbase, rend, gbase, w, enq);
    // per item: the remaining arcs with the whole wavefront, then the path
    // counts and target levels of its lanes
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const int ld = t * SUB;
      const ull mt = read_lane64(mask, ld);
      if (mt == 0ull) {  // slot past the end of the list (or an empty item)
        if (lane == 0 && i0 + (uint64_t)t < count) S.imask[base + i0 + t] = 0ull;
        continue;
      }
      const uint32_t itt = read_lane(it, ld);
      const uint32_t gt = read_lane(g, ld);
      const uint64_t gbt = read_lane64(gbase, ld);
      const int64_t F1 = (int64_t)read_lane64((ull)f1, ld), E1 = (int64_t)read_lane64((ull)d1, ld);
      const int64_t F0 = (int64_t)read_lane64((ull)f0, ld), E0 = (int64_t)read_lane64((ull)e0, ld);
      const uint64_t deg = (uint64_t)((int64_t)read_lane64((ull)e1, ld) - E0);
      c_it += 1;
      c_ia += deg;
      if (pull) {  // a level found bottom-up was counted there
        c_v += (uint64_t)__popcll(mt);
        c_a += (uint64_t)__popcll(mt) * deg;
      }
      for (int64_t e = F0 + SUB; e < F1; e += kLanes) {
        const int64_t my = e + lane;
        uint32_t uu = 0;
        ull pp = 0ull, pd = 0ull;
        if (my < F1) {
          uu = (uint32_t)G.icol[my];
          pp = rec[gbt + uu].fr[kp] & mt;
          if (pp != 0ull) pd = rec[gbt + uu].dn;
        }
        ull a1[1] = {acc[t]};
        bool l1[1] = {lov[t]};
        pull_slots<1>(S, gbt, uu, pp, lane, a1, l1, l1, c_d);
        acc[t] = a1[0];
        lov[t] = l1[0];
        ull d1[1] = {0ull};
        or_slots<1>(pp & pd, d1);
        dnacc[t] |= d1[0];
      }
      for (int64_t e = E0 + SUB; e < E1; e += kLanes) {
        const int64_t my = e + lane;
        uint32_t ww = 0;
        bool eq = false;
        if (my < E1) {
          ww = (uint32_t)G.col[my];
          const MaskRec &R = rec[gbt + ww];
          const ull dd = mt & ~(R.vis | R.fr[kc] | R.fr[kn]);
          if (dd != 0ull) eq = (atomicOr(&rec[gbt + ww].fr[kn], dd) == 0ull);
        }
        append_chunk(S, stage, nst, next_cnt, nbase, rend, gbt, ww, eq);
      }
      // the item's lanes for the backward: all of them for exports, else
      // those where v is a target or lies below one (a target's dependency
      // reads psi nowhere else)
      if (!pull) {  // found bottom-up: its marks are in the record already
        if (lane == 0) S.imask[base + i0 + t] = S.keep_all ? mt : (mt & rec[itt].dn);
        continue;
      }
      const bool act = (mt >> lane) & 1ull;
      const bool is_tgt = (int32_t)read_lane((uint32_t)tg, ld) >= 0;
      if (is_tgt && lane == 0) atomicMin(S.tmin, (uint32_t)level);
      const ull dnt = dnacc[t] | (is_tgt ? mt : 0ull);
      if (lane == 0) {
        if (dnt != 0ull) rec[itt].dn = rec[itt].dn | dnt;
        S.imask[base + i0 + t] = S.keep_all ? mt : dnt;
      }
      if (level > 0) {
        if (act) S.sig[(uint64_t)itt * kLanes + lane] = acc[t];
        if (lov[t]) {
          ovf = true;
          atomicOr(&S.ovl[gt], 1ull << lane);
        }
      }
    }
  }
  flush_stage(S, stage, nst, next_cnt, nbase, rend);
  const int ck[5] = {C_FWD_VPAIRS, C_FWD_APAIRS, C_FWD_DPAIRS, C_FWD_ITEMS, C_FWD_IARCS};
  const uint64_t cv[5] = {c_v, c_a, c_d, c_it, c_ia};
  flush_wave_counters<BLOCK, 5>(S.ctr, S.ctr_slots, ck, cv, ovf, S.flags);
}

// Push form of the path counts: sigma_b(w) += sigma_b(v) for every DAG arc
// (v, w) of lane b, one 64-bit atomic add per (lane, DAG arc).  The chunk
// holds the out-arcs of up to K items (slot t = arc lane / (64 / K));
// `push` on an arc lane holds the lanes for which that arc is a DAG arc, sv[t]
// is this lane's path count at item t and dn[t] (wave-uniform) the item's
// lanes that are a target or lie below one, which follow the count to the
// head.  Adds of up to eight arcs are issued before their results are
// checked; an add whose result wraps means the exact count exceeds 2^64 - 1
// (every addend is nonnegative, so the running sum crosses 2^64 once).
template <int K>
static __device__ __forceinline__ void push_slots(const BatchState &S, uint64_t gbase, uint32_t w, ull push,
                                                  int lane, const ull (&sv)[K], const ull (&dn)[K], bool &ovf,
                                                  uint64_t &dag_pairs) {
  constexpr int SUB = kLanes / K;
  ull bits = __ballot(push != 0ull);
  while (bits != 0ull) {
    int j[8];
    int c = 0;
    for (; c < 8 && bits != 0ull; ++c) {
      j[c] = __ffsll((long long)bits) - 1;
      bits &= bits - 1ull;
    }
    ull old[8], add[8];
    uint64_t gq8[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      old[q] = 0ull;
      add[q] = 0ull;
      gq8[q] = 0;
      if (q < c) {
        const uint32_t wq = read_lane(w, j[q]);
        const ull dq = read_lane64(push, j[q]);
        const uint64_t gq = read_lane64(gbase, j[q]);
        const int slot = j[q] / SUB;
        ull x = sv[0], dnq = dn[0];
#pragma unroll
        for (int t = 1; t < K; ++t)
          if (slot == t) {
            x = sv[t];
            dnq = dn[t];
          }
        dag_pairs += (uint64_t)__popcll(dq);  // wave-uniform
        gq8[q] = gq + wq;
        if ((dq >> lane) & 1ull) {
          add[q] = x;
          old[q] = atomicAdd(&S.sig[(gq + wq) * kLanes + lane], x);
        }
        // the head's lanes below a target on this arc (one atomic per arc)
        const ull dd = dnq & dq;
        if (dd != 0ull && lane == 0) atomicOr(&S.rec[gq + wq].dn, dd);
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (q < c && old[q] + add[q] < old[q]) {
        ovf = true;
        atomicOr(&S.ovl[(uint32_t)(gq8[q] / (uint64_t)S.n)], 1ull << lane);
      }
  }
}

// One BFS level of the batched forward pass with pushed path counts (the
// alternative to k_fwd_level's pull; same results bit for bit, since the
// counts are exact integer sums).  For every item (g, v, mask) on `level`:
// sigma_b(v) is final (pushed by the level before, or pulled by k_bu_level
// when this level was found bottom-up); every out-arc (v, w) whose head is
// not settled on a level <= `level` for lane b of mask is a DAG arc of lane
// b: w is flagged for level+1 (one atomicOr per arc, the first flagger
// appends it) and sigma_b(v) is added into sigma_b(w).  No in-arc is read.
// Path-count rows must start at zero on every lane (k_batch_cleanup resets
// the lanes a batch settled).
template <int BLOCK, int K>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_fwd_push(DevGraph G,
                                                                                                BatchState S,
                                                                                                int level) {
  constexpr int SUB = kLanes / K;
  const uint64_t n = (uint64_t)S.n;
  const int P = S.P;
  const PartView pv = part_view<BLOCK>(P);
  const uint64_t base = S.off[(uint64_t)level * P + pv.p];
  const uint64_t count = S.cnt[(uint64_t)level * P + pv.p];
  const uint64_t nbase = base + count;
  const uint64_t rend = (uint64_t)(pv.p + 1) * S.capP;
  if (pv.thread == 0) S.off[(uint64_t)(level + 1) * P + pv.p] = nbase;
  if (nbase > rend) return;  // capacity exceeded (workgroup-uniform test): the batch is redone
  const int lane = lane_id();
  const int sl = lane % SUB;
  MaskRec *rec = S.rec;
  const int kc = level & 3, kn = (level + 1) & 3, ko = (level + 2) & 3;
  if (level >= 2) {  // retire the masks of level-2
    const uint64_t pb = S.off[(uint64_t)(level - 2) * P + pv.p];
    const uint64_t pc = S.cnt[(uint64_t)(level - 2) * P + pv.p];
    for (uint64_t i = pv.thread; i < pc; i += pv.nthreads) rec[S.items[pb + i]].fr[ko] = 0ull;
  }
  uint64_t prev = 0;
  if (level >= 1)
    for (int p = 0; p < P; ++p) prev += S.cnt[(uint64_t)(level - 1) * P + p];
  uint64_t cur = 0;
  for (int p = 0; p < P; ++p) cur += S.cnt[(uint64_t)level * P + p];
  const bool own = !bottom_up_rule(S.bu_den, level, prev, S.gused, S.n);  // found top-down
  const bool disc = !bottom_up_rule(S.bu_den, level + 1, cur, S.gused, S.n);

  uint64_t c_v = 0, c_a = 0, c_d = 0, c_it = 0, c_ia = 0;  // wave-uniform counters
  bool ovf = false;
  const uint64_t step = pv.nwaves * (uint64_t)K;
  uint32_t *next_cnt = &S.cnt[(uint64_t)(level + 1) * P + pv.p];
  __shared__ uint32_t stage_all[(BLOCK / 64) * kStage];
  uint32_t *stage = stage_all + (threadIdx.x >> 6) * kStage;
  int nst = 0;
  uint64_t ii = pv.wave * (uint64_t)K + (uint64_t)(lane / SUB);  // this lane's item
  uint32_t it_next = ii < count ? S.items[base + ii] : 0u;
  for (uint64_t i0 = pv.wave * (uint64_t)K; i0 < count; i0 += step, ii += step) {
    const bool has = ii < count;
    const uint32_t it = it_next;
    if (ii + step < count) it_next = S.items[base + ii + step];
    const uint32_t g = (uint32_t)(it / n);
    const uint32_t v = (uint32_t)(it - (uint64_t)g * n);
    const uint64_t gbase = (uint64_t)g * n;
    ull mask = 0ull, dnr = 0ull;
    int64_t e0 = 0, e1 = 0;
    int32_t tg = -1;
    if (has) {
      mask = rec[it].fr[kc];
      dnr = rec[it].dn;
      e0 = G.rp[v];
      e1 = G.rp[v + 1];
      if (own) tg = S.tgt_of[v];
    }
    const int64_t d1 = disc ? e1 : e0;  // end of the out-arcs to scan
    if (has && sl == 0 && own) rec[it].vis = rec[it].vis | mask;
    // per slot: the item's lanes, their marks, and this lane's path count
    ull mt[K], dn[K], sv[K];
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const int ld = t * SUB;
      mt[t] = read_lane64(mask, ld);
      const bool is_tgt = (int32_t)read_lane((uint32_t)tg, ld) >= 0;
      dn[t] = (read_lane64(dnr, ld) | (is_tgt ? mt[t] : 0ull)) & mt[t];
      sv[t] = ((mt[t] >> lane) & 1ull) ? S.sig[(uint64_t)read_lane(it, ld) * kLanes + lane] : 0ull;
    }
    // first chunk of every slot's out-arcs: heads, their records, the flags
    const int64_t mo = e0 + sl;
    uint32_t w = 0;
    ull push = 0ull;
    bool enq = false;
    if (mo < d1) {
      w = (uint32_t)G.col[mo];
      const MaskRec &R = rec[gbase + w];
      const ull settled = R.vis | R.fr[kc];
      push = mask & ~settled;  // the DAG lanes of this arc
      const ull dag = push & ~R.fr[kn];  // lanes already flagged by another wavefront need no atomic
      if (dag != 0ull) enq = (atomicOr(&rec[gbase + w].fr[kn], dag) == 0ull);
    }
    push_slots<K>(S, gbase, w, push, lane, sv, dn, ovf, c_d);
    append_chunk(S, stage, nst, next_cnt, nbase, rend, gbase, w, enq);
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const int ld = t * SUB;
      const ull m = mt[t];
      if (m == 0ull) {  // slot past the end of the list (or an empty item)
        if (lane == 0 && i0 + (uint64_t)t < count) S.imask[base + i0 + t] = 0ull;
        continue;
      }
      const uint32_t itt = read_lane(it, ld);
      const uint64_t gbt = read_lane64(gbase, ld);
      const int64_t E0 = (int64_t)read_lane64((ull)e0, ld), E1 = (int64_t)read_lane64((ull)d1, ld);
      const uint64_t deg = (uint64_t)((int64_t)read_lane64((ull)e1, ld) - E0);
      c_it += 1;
      c_ia += deg;
      if (own) {  // a level found bottom-up was counted and marked there
        c_v += (uint64_t)__popcll(m);
        c_a += (uint64_t)__popcll(m) * deg;
        const bool is_tgt = (int32_t)read_lane((uint32_t)tg, ld) >= 0;
        if (is_tgt && lane == 0) {
          atomicMin(S.tmin, (uint32_t)level);
          rec[itt].dn = rec[itt].dn | m;
        }
      }
      if (lane == 0) S.imask[base + i0 + t] = S.keep_all ? m : dn[t];
      ull s1[1] = {sv[t]}, d1m[1] = {dn[t]};
      for (int64_t e = E0 + SUB; e < E1; e += kLanes) {
        const int64_t my = e + lane;
        uint32_t ww = 0;
        ull pp = 0ull;
        bool eq = false;
        if (my < E1) {
          ww = (uint32_t)G.col[my];
          const MaskRec &R = rec[gbt + ww];
          pp = m & ~(R.vis | R.fr[kc]);
          const ull dd = pp & ~R.fr[kn];
          if (dd != 0ull) eq = (atomicOr(&rec[gbt + ww].fr[kn], dd) == 0ull);
        }
        push_slots<1>(S, gbt, ww, pp, lane, s1, d1m, ovf, c_d);
        append_chunk(S, stage, nst, next_cnt, nbase, rend, gbt, ww, eq);
      }
    }
  }
  flush_stage(S, stage, nst, next_cnt, nbase, rend);
  const int ck[5] = {C_FWD_VPAIRS, C_FWD_APAIRS, C_FWD_DPAIRS, C_FWD_ITEMS, C_FWD_IARCS};
  const uint64_t cv[5] = {c_v, c_a, c_d, c_it, c_ia};
  flush_wave_counters<BLOCK, 5>(S.ctr, S.ctr_slots, ck, cv, ovf, S.flags);
}

// 64-bit lane shuffle (ds_bpermute on both halves).
static __device__ __forceinline__ ull shfl64(ull x, int src) {
  const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)x, src);
  const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(x >> 32), src);
  return ((ull)hi << 32) | lo;
}

// One BFS level found bottom-up (direction-optimizing BFS, here over 64
// sources at once): every (g, w) of the batch with in-arcs and with lanes
// not yet settled scans its in-arcs (u, w); lanes b of u's previous-level
// mask that are unsettled at w are DAG arcs of w on this level, so one scan
// both finds the level's lanes of w and pulls their path counts (a lane is
// on the level iff some in-arc delivered a count to it).  No atomics on the
// masks; (g, w) is appended to the level's list if it gained any lane.
// Runs before the top-down kernel of the same level, and only when
// bottom_up_rule holds for the level.  The unsettled pairs of a 64-vertex
// block are taken K at a time, 64 / K lanes each for their first in-arcs.
template <int BLOCK, int K>
__global__ __launch_bounds__(BLOCK) void k_bu_level(DevGraph G, BatchState S, int level) {
  constexpr int SUB = kLanes / K;
  const uint64_t n = (uint64_t)S.n;
  const int P = S.P;
  uint64_t prev = 0;
  for (int p = 0; p < P; ++p) prev += S.cnt[(uint64_t)(level - 1) * P + p];
  if (!bottom_up_rule(S.bu_den, level, prev, S.gused, S.n)) return;
  const PartView pv = part_view<BLOCK>(P);
  const uint64_t base = S.off[(uint64_t)level * P + pv.p];
  const uint64_t rend = (uint64_t)(pv.p + 1) * S.capP;
  if (base > rend) return;  // capacity exceeded earlier (workgroup-uniform test): the batch is redone
  const int lane = lane_id();
  const int slot = lane / SUB, sl = lane % SUB;
  MaskRec *rec = S.rec;
  const int kc = level & 3, kp = (level + 3) & 3;
  uint32_t *cnt_here = &S.cnt[(uint64_t)level * P + pv.p];
  __shared__ uint32_t stage_all[(BLOCK / 64) * kStage];
  uint32_t *stage = stage_all + (threadIdx.x >> 6) * kStage;
  int nst = 0;
  uint64_t c_v = 0, c_a = 0, c_d = 0;
  bool ovf = false;
  // groups p, p + P, ... below gused belong to this partition
  const uint64_t ngp = S.gused > pv.p ? (uint64_t)(S.gused - pv.p + P - 1) / (uint64_t)P : 0;
  const uint64_t nvb = (n + 63) / 64;
  for (uint64_t b = pv.wave; b < ngp * nvb; b += pv.nwaves) {
    const uint64_t gl = b / nvb;
    const uint32_t g = (uint32_t)(pv.p + gl * (uint64_t)P);
    const uint64_t gbase = (uint64_t)g * n;
    const uint64_t w0 = (b - gl * nvb) * 64;
    const uint64_t w = w0 + lane;
    const ull act_lanes = (g + 1 == (uint32_t)S.gused) ? S.last_lanes : ~0ull;
    int64_t f0 = 0, f1 = 0;
    ull uns = 0ull;
    if (w < n) {
      f0 = G.irp[w];
      f1 = G.irp[w + 1];
      if (f1 > f0) uns = act_lanes & ~rec[gbase + w].vis;
    }
    ull cm = __ballot(uns != 0ull);
    while (cm != 0ull) {
      // the next K candidates of the block, one per slot
      int jc[K];
#pragma unroll
      for (int t = 0; t < K; ++t) {
        jc[t] = cm != 0ull ? __ffsll((long long)cm) - 1 : -1;
        if (cm != 0ull) cm &= cm - 1ull;
      }
      int js = jc[0];
#pragma unroll
      for (int t = 1; t < K; ++t)
        if (slot == t) js = jc[t];
      // the shuffles run on every lane: a permute reads nothing from a lane
      // that is switched off, and the candidate's own lane may sit in a slot
      // that has no candidate this step
      const int src = js < 0 ? 0 : js;
      const ull un_src = shfl64(uns, src);
      const int64_t F0 = (int64_t)shfl64((ull)f0, src);
      const int64_t F1_src = (int64_t)shfl64((ull)f1, src);
      const ull un = js < 0 ? 0ull : un_src;
      const int64_t F1 = js < 0 ? F0 : F1_src;
      // first chunk of every slot's in-arcs
      const int64_t mi = F0 + sl;
      uint32_t u = 0;
      ull pfr = 0ull, pdn = 0ull;
      if (mi < F1) {
        u = (uint32_t)G.icol[mi];
        pfr = rec[gbase + u].fr[kp];
        pdn = rec[gbase + u].dn;
      }
      const ull pm = pfr & un;
      ull acc[K];
      bool lov[K], hit[K];
#pragma unroll
      for (int t = 0; t < K; ++t) {
        acc[t] = 0ull;
        lov[t] = false;
        hit[t] = false;
      }
      pull_slots<K, true>(S, gbase, u, pm, lane, acc, lov, hit, c_d);
      ull dnacc[K];
#pragma unroll
      for (int t = 0; t < K; ++t) dnacc[t] = 0ull;
      or_slots<K>(pm & pdn, dnacc);
#pragma unroll
      for (int t = 0; t < K; ++t) {
        if (jc[t] < 0) continue;
        const ull ut = read_lane64(uns, jc[t]);
        const int64_t G0 = (int64_t)read_lane64((ull)f0, jc[t]), G1 = (int64_t)read_lane64((ull)f1, jc[t]);
        for (int64_t e = G0 + SUB; e < G1; e += kLanes) {
          const int64_t my = e + lane;
          uint32_t uu = 0;
          ull pp = 0ull, pd = 0ull;
          if (my < G1) {
            uu = (uint32_t)G.icol[my];
            pp = rec[gbase + uu].fr[kp] & ut;
            pd = rec[gbase + uu].dn;
          }
          ull a1[1] = {acc[t]};
          bool l1[1] = {lov[t]}, h1[1] = {hit[t]};
          pull_slots<1, true>(S, gbase, uu, pp, lane, a1, l1, h1, c_d);
          acc[t] = a1[0];
          lov[t] = l1[0];
          hit[t] = h1[0];
          ull d1[1] = {0ull};
          or_slots<1>(pp & pd, d1);
          dnacc[t] |= d1[0];
        }
        const ull nm = __ballot(hit[t]);  // lanes of w on this level
        if (nm == 0ull) continue;
        const uint32_t wt = (uint32_t)(w0 + (uint64_t)jc[t]);
        const uint32_t it = (uint32_t)(gbase + wt);
        const bool act = (nm >> lane) & 1ull;
        const int64_t e0 = G.rp[wt], e1 = G.rp[wt + 1];
        const int32_t tg = S.tgt_of[wt];
        if (act) S.sig[(uint64_t)it * kLanes + lane] = acc[t];
        if (lov[t]) {
          ovf = true;
          atomicOr(&S.ovl[g], 1ull << lane);
        }
        const ull dnt = (dnacc[t] & nm) | (tg >= 0 ? nm : 0ull);
        if (lane == 0) {
          rec[it].fr[kc] = nm;
          rec[it].vis = rec[it].vis | nm;
          if (dnt != 0ull) rec[it].dn = rec[it].dn | dnt;
        }
        c_v += (uint64_t)__popcll(nm);
        c_a += (uint64_t)__popcll(nm) * (uint64_t)(e1 - e0);
        if (tg >= 0 && lane == 0) atomicMin(S.tmin, (uint32_t)level);
        append_chunk(S, stage, nst, cnt_here, base, rend, gbase, wt, lane == 0);
      }
    }
  }
  flush_stage(S, stage, nst, cnt_here, base, rend);
  const int ck[3] = {C_FWD_VPAIRS, C_FWD_APAIRS, C_FWD_DPAIRS};
  const uint64_t cv[3] = {c_v, c_a, c_d};  // wave-uniform
  flush_wave_counters<BLOCK, 3>(S.ctr, S.ctr_slots, ck, cv, ovf, S.flags);
}

// Sum of psi_b(w) over the out-arcs held by one chunk of lanes whose head w
// is a shortest-path-DAG successor for lane b (d = lanes of that arc); the
// chunk holds the arcs of up to K items, 64 / K lanes each, and an arc adds
// into its item's accumulator.  Bits are taken in lane order, which is arc
// order within an item, so every item's sum runs in arc order whatever K is.
// Row loads of up to eight successors are issued before any is consumed.
template <int K>
static __device__ __forceinline__ void push_sum_slots(const BatchState &S, uint64_t gbase, uint32_t w, ull d,
                                                      int lane, double (&acc)[K], uint64_t &dag_pairs) {
  constexpr int SUB = kLanes / K;
  ull bits = __ballot(d != 0ull);
  while (bits != 0ull) {
    int j[8];
    int c = 0;
    for (; c < 8 && bits != 0ull; ++c) {
      j[c] = __ffsll((long long)bits) - 1;
      bits &= bits - 1ull;
    }
    double x[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      x[q] = 0.0;
      if (q < c) {
        const uint32_t wq = read_lane(w, j[q]);
        const ull dq = read_lane64(d, j[q]);
        const uint64_t gq = read_lane64(gbase, j[q]);
        dag_pairs += (uint64_t)__popcll(dq);  // wave-uniform
        if ((dq >> lane) & 1ull) x[q] = S.psi[(gq + wq) * kLanes + lane];
      }
    }
    // adding 0.0 for a lane off the DAG leaves its sum unchanged
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (q < c) {
        const int slot = j[q] / SUB;
#pragma unroll
        for (int t = 0; t < K; ++t)
          if (slot == t) acc[t] += x[q];
      }
    }
  }
}

// One level of the backward pass, Eq.(4) read as
//   delta(v) = sigma(v) * sum_{w: v in P(w)} psi(w),  psi(w) = (1 + delta(w)) / sigma(w),
// so psi(v) = 1/sigma(v) + sum psi(w).  Successor w of v is on the DAG for
// lane b iff w sits on level+1 for b, read from the level-tagged table the
// previous (deeper) launch wrote.  Only the lanes the forward kept in the
// item's mask are computed -- those where v is a target or lies below one
// (no target's dependency reads psi anywhere else) -- and target vertices
// report delta on their lanes.  No atomics: every sum runs
// in arc order, so results are bit-reproducible.  A wavefront takes K items
// per step, their first 64 / K out-arcs in one chunk of lanes (as in the
// forward kernel), then longer out-arc lists 64 at a time.
template <int BLOCK, int K>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(7, 8))) void k_bwd_level(DevGraph G,
                                                                                                 BatchState S,
                                                                                                 int level, int ntgt,
                                                                                                 int full) {
  constexpr int SUB = kLanes / K;
  const uint64_t n = (uint64_t)S.n;
  const uint64_t GN = (uint64_t)S.G * n;
  const int P = S.P;
  const PartView pv = part_view<BLOCK>(P);
  const uint64_t base = S.off[(uint64_t)level * P + pv.p];
  const uint64_t count = S.cnt[(uint64_t)level * P + pv.p];
  if (base + count > (uint64_t)(pv.p + 1) * S.capP) return;
  const int lane = lane_id();
  const int sl = lane % SUB;
  const LevMask *bt_in = S.bt + (uint64_t)((level + 1) & 1) * GN;
  LevMask *bt_out = S.bt + (uint64_t)(level & 1) * GN;
  const uint32_t E = S.epoch;
  uint64_t c_v = 0, c_a = 0, c_d = 0, c_it = 0, c_ia = 0;  // wave-uniform counters
  const uint64_t step = pv.nwaves * (uint64_t)K;
  uint64_t ii = pv.wave * (uint64_t)K + (uint64_t)(lane / SUB);  // this lane's item
  // the next step's ids and masks are loaded while this one is processed
  uint32_t it_next = ii < count ? S.items[base + ii] : 0u;
  ull mask_next = ii < count ? S.imask[base + ii] : 0ull;
  for (uint64_t i0 = pv.wave * (uint64_t)K; i0 < count; i0 += step, ii += step) {
    const uint32_t it = it_next;
    const ull mask = mask_next;
    if (ii + step < count) {
      it_next = S.items[base + ii + step];
      mask_next = S.imask[base + ii + step];
    }
    const uint32_t g = (uint32_t)(it / n);
    const uint32_t v = (uint32_t)(it - (uint64_t)g * n);
    const uint64_t gbase = (uint64_t)g * n;
    int32_t tg = -1;
    int64_t e0 = 0, e1 = 0;
    if (mask != 0ull) {
      tg = S.tgt_of[v];
      e0 = G.rp[v];
      e1 = G.rp[v + 1];
    }
    // lanes of each item that need psi here, and their path counts
    ull emv[K], my_em = 0ull;
    ull sg[K];
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const int ld = t * SUB;
      const ull mt = read_lane64(mask, ld);
      emv[t] = 0ull;
      sg[t] = 1ull;
      if (mt == 0ull) continue;
      // the forward kept only the lanes that need psi here (all of them for
      // exports): those where v is a target or lies below one
      const bool need = (mt >> lane) & 1ull;
      emv[t] = __ballot(need);
      if (need) sg[t] = S.sig[(uint64_t)read_lane(it, ld) * kLanes + lane];
    }
#pragma unroll
    for (int t = 0; t < K; ++t)
      if (lane / SUB == t) my_em = emv[t];
    // first chunk of every slot's out-arcs
    const int64_t mo = e0 + sl;
    uint32_t w = 0;
    ull d = 0ull;
    if (my_em != 0ull && mo < e1) {
      w = (uint32_t)G.col[mo];
      const LevMask tw = bt_in[gbase + w];
      const ull mw = (tw.lev == (uint32_t)(level + 1) && tw.epoch == E) ? tw.mask : 0ull;
      d = my_em & mw;
    }
    double acc[K];
#pragma unroll
    for (int t = 0; t < K; ++t) acc[t] = 0.0;
    push_sum_slots<K>(S, gbase, w, d, lane, acc, c_d);
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const ull em = emv[t];
      if (em == 0ull) continue;
      const int ld = t * SUB;
      const uint32_t itt = read_lane(it, ld);
      const uint32_t gt = read_lane(g, ld);
      const uint64_t gbt = read_lane64(gbase, ld);
      const int64_t E0 = (int64_t)read_lane64((ull)e0, ld), E1 = (int64_t)read_lane64((ull)e1, ld);
      // remaining out-arcs, 64 at a time, still in arc order
      for (int64_t e = E0 + SUB; e < E1; e += kLanes) {
        const int64_t my = e + lane;
        uint32_t ww = 0;
        ull dd = 0ull;
        if (my < E1) {
          ww = (uint32_t)G.col[my];
          const LevMask tw = bt_in[gbt + ww];
          const ull mw = (tw.lev == (uint32_t)(level + 1) && tw.epoch == E) ? tw.mask : 0ull;
          dd = em & mw;
        }
        double a1[1] = {acc[t]};
        push_sum_slots<1>(S, gbt, ww, dd, lane, a1, c_d);
        acc[t] = a1[0];
      }
      const int32_t tgt = (int32_t)read_lane((uint32_t)tg, ld);
      if ((em >> lane) & 1ull) {
        const double s = (double)sg[t];
        const double dl = s * acc[t];
        S.psi[(uint64_t)itt * kLanes + lane] = acc[t] + 1.0 / s;
        if (S.dout) S.dout[(uint64_t)itt * kLanes + lane] = dl;
        if (tgt >= 0 && tgt < ntgt)
          S.res[((uint64_t)tgt * S.G + gt) * kLanes + lane] = (level > 0) ? dl : 0.0;
      }
      if (lane == 0) {
        LevMask o;
        o.mask = em;
        o.lev = (uint32_t)level;
        o.epoch = E;
        bt_out[itt] = o;
      }
      c_v += (uint64_t)__popcll(em);
      c_a += (uint64_t)__popcll(em) * (uint64_t)(E1 - E0);
      c_it += 1;
      c_ia += (uint64_t)(E1 - E0);
    }
  }
  const int ck[5] = {C_BWD_VPAIRS, C_BWD_APAIRS, C_BWD_DPAIRS, C_BWD_ITEMS, C_BWD_IARCS};
  const uint64_t cv[5] = {c_v, c_a, c_d, c_it, c_ia};
  flush_wave_counters<BLOCK, 5>(S.ctr, S.ctr_slots, ck, cv, false, S.flags);
}

// Reset what the batch touched: the masks of every item and, when the path
// counts were pushed (added into), the counts of every lane the batch
// settled, so the next batch's adds start from zero.  (Pulled counts need no
// reset: every lane's count is written before anything reads it, and only
// lanes named by a mask are ever read.)  A wavefront per item, lanes over
// the 64 counts of its row; an item repeated on several levels clears the
// row again or finds the record already cleared, and either way every
// settled lane is zeroed by the first wavefront that read the record.
__global__ void k_batch_cleanup(BatchState S, PartTotals tot) {
  const int lane = lane_id();
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (int p = 0; p < S.P; ++p) {
    uint64_t total = tot.t[p];
    if (total > S.capP) total = S.capP;
    const uint32_t *items = S.items + (uint64_t)p * S.capP;
    for (uint64_t i = wave; i < total; i += nwaves) {
      const uint32_t it = items[i];
      MaskRec &R = S.rec[it];
      if (S.push) {
        const ull vis = R.vis;
        if ((vis >> lane) & 1ull) S.sig[(uint64_t)it * kLanes + lane] = 0ull;
      }
      if (lane < 6) {
        if (lane == 0) R.vis = 0ull;
        else if (lane == 1) R.dn = 0ull;
        else R.fr[lane - 2] = 0ull;
      }
    }
  }
}

// Verification export of one level: per lane with a slot, distance = level,
// sigma and delta from the state rows.
__global__ void k_batch_export(BatchState S, int level, uint64_t begin, uint64_t count,
                               const int32_t *lane_slot, uint64_t *dist, ull *sigma, double *delta,
                               int64_t k) {
  const uint64_t n = (uint64_t)S.n;
  const int lane = lane_id();
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  if (begin + count > S.cap) return;
  for (uint64_t i = wave; i < count; i += nwaves) {
    const uint32_t it = S.items[begin + i];  // begin: absolute position (partition region + level offset)
    const uint32_t g = (uint32_t)(it / n);
    const uint32_t v = (uint32_t)(it - (uint64_t)g * n);
    const ull mask = S.imask[begin + i];
    if (!((mask >> lane) & 1ull)) continue;
    const int32_t slot = lane_slot[g * kLanes + lane];
    if (slot < 0 || slot >= k) continue;
    const uint64_t o = (uint64_t)slot * n + v;
    dist[o] = (uint64_t)level;
    sigma[o] = S.sig[(uint64_t)it * kLanes + lane];
    if (delta && S.dout) delta[o] = S.dout[(uint64_t)it * kLanes + lane];
  }
}

// --------------------------------------------------------------- plain

__global__ void k_plain_init(PlainState P, int32_t s) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    P.d[s] = 0;
    P.sig[s] = 1ull;
    P.queue[0] = s;
    P.cnt[0] = 1u;
    P.off[0] = 0ull;
  }
}

// One BFS level from a single source: a wavefront per frontier vertex,
// lanes over its out-arcs; the first lane to claim a vertex appends it
// (ballot + mbcnt compaction, one queue atomic per wavefront).
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_plain_fwd(DevGraph G, PlainState P, int level) {
  const uint64_t base = P.off[level];
  const uint64_t count = P.cnt[level];
  const uint64_t nbase = base + count;
  if (blockIdx.x == 0 && threadIdx.x == 0) P.off[level + 1] = nbase;
  if (nbase > (uint64_t)P.n) return;
  const int lane = lane_id();
  uint64_t c_v = 0, c_a = 0, c_d = 0;
  bool ovf = false;
  const uint64_t wave = ((uint64_t)blockIdx.x * BLOCK + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * BLOCK) >> 6;
  for (uint64_t i = wave; i < count; i += nwaves) {
    const int32_t v = P.queue[base + i];
    const ull sv = P.sig[v];
    const int64_t e0 = G.rp[v], e1 = G.rp[v + 1];
    if (lane == 0) {
      c_v += 1;
      c_a += (uint64_t)(e1 - e0);
    }
    for (int64_t e = e0; e < e1; e += 64) {
      const int64_t my = e + lane;
      bool enq = false, dag = false;
      int32_t w = 0;
      if (my < e1) {
        w = G.col[my];
        int32_t dw = P.d[w];
        if (dw < 0) {
          const int32_t o = atomicCAS(&P.d[w], -1, level + 1);
          if (o == -1) {
            enq = true;
            dw = level + 1;
          } else {
            dw = o;
          }
        }
        dag = (dw == level + 1);
        if (dag) {
          const ull o = atomicAdd(&P.sig[w], sv);
          if (o + sv < o) ovf = true;
        }
      }
      c_d += dag ? 1 : 0;
      const ull eb = __ballot(enq);
      if (eb != 0ull) {
        uint32_t p0 = 0;
        if (lane == 0) p0 = atomicAdd(&P.cnt[level + 1], (uint32_t)__popcll(eb));
        p0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)p0);
        if (enq) {
          const uint64_t p = nbase + p0 + (uint64_t)lanes_below(eb);
          if (p < (uint64_t)P.n) P.queue[p] = w;
        }
      }
    }
  }
  flush_counters<BLOCK>(P.ctr, P.ctr_slots, C_FWD_VPAIRS, c_v, c_a, c_d, ovf, P.flags);
}

// One backward level from a single source: lanes over out-arcs gather psi
// of successors on level+1; the wavefront sum is a fixed shuffle tree.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_plain_bwd(DevGraph G, PlainState P, int level, int32_t target,
                                                     int only_target) {
  const uint64_t base = P.off[level];
  const uint64_t count = P.cnt[level];
  if (base + count > (uint64_t)P.n) return;
  const int lane = lane_id();
  uint64_t c_v = 0, c_a = 0, c_d = 0;
  const uint64_t wave = ((uint64_t)blockIdx.x * BLOCK + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * BLOCK) >> 6;
  for (uint64_t i = wave; i < count; i += nwaves) {
    const int32_t v = P.queue[base + i];
    if (only_target && v != target) continue;
    const int64_t e0 = G.rp[v], e1 = G.rp[v + 1];
    double acc = 0.0;
    for (int64_t e = e0; e < e1; e += 64) {
      const int64_t my = e + lane;
      if (my < e1) {
        const int32_t w = G.col[my];
        if (P.d[w] == level + 1) {
          acc += P.psi[w];
          c_d += 1;
        }
      }
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) {
      const double s = (double)P.sig[v];
      P.psi[v] = acc + 1.0 / s;
      P.dout[v] = s * acc;
      c_v += 1;
      c_a += (uint64_t)(e1 - e0);
    }
  }
  flush_counters<BLOCK>(P.ctr, P.ctr_slots, C_BWD_VPAIRS, c_v, c_a, c_d, false, P.flags);
}

__global__ void k_plain_cleanup(PlainState P, uint64_t total) {
  if (total > (uint64_t)P.n) total = (uint64_t)P.n;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const int32_t v = P.queue[i];
    P.d[v] = -1;
    P.sig[v] = 0ull;
  }
}

__global__ void k_plain_export(PlainState P, uint64_t *dist, ull *sigma, double *delta) {
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < (uint64_t)P.n;
       v += (uint64_t)gridDim.x * blockDim.x) {
    const int32_t d = P.d[v];
    if (dist) dist[v] = d < 0 ? ~0ull : (uint64_t)d;
    if (sigma) sigma[v] = d < 0 ? 0ull : P.sig[v];
    if (delta) delta[v] = d < 0 ? 0.0 : P.dout[v];
  }
}

// --------------------------------------------------------- reachability

__global__ void k_reach_init(uint32_t *bitmap, int32_t *q, uint32_t *qn, int32_t root) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    bitmap[root >> 5] |= 1u << (root & 31);
    q[0] = root;
    *qn = 1u;
  }
}

// Adds a wavefront's per-lane counts into *dst with one atomic.
static __device__ __forceinline__ void wave_add_u64(uint64_t *dst, uint64_t x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  if (lane_id() == 0 && x != 0) atomicAdd((unsigned long long *)dst, (unsigned long long)x);
}

// One BFS level on a CSR, weights ignored: a wavefront per frontier vertex,
// lanes over arcs, first setter of a bit appends the vertex.  Every append
// adds the vertex's arc count (its row in this CSR) to *qout_a, the arcs the
// next level scans top-down; a level whose frontier has at least bu_arcs of
// them is left to k_reach_bu.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_reach_level(const int64_t *rp, const int32_t *col, uint32_t *bitmap,
                                                       const int32_t *qin, const uint32_t *qin_n,
                                                       const uint64_t *qin_a, int32_t *qout, uint32_t *qout_n,
                                                       uint64_t *qout_a, uint8_t *lev, int level,
                                                       uint64_t bu_arcs) {
  const int lane = lane_id();
  const uint32_t count = *qin_n;
  if (*qin_a >= bu_arcs) return;  // found bottom-up (the same test in both kernels)
  uint64_t arcs = 0;
  const uint64_t wave = ((uint64_t)blockIdx.x * BLOCK + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * BLOCK) >> 6;
  __shared__ uint32_t st_all[(BLOCK / 64) * kStage];
  uint32_t *stg = st_all + (threadIdx.x >> 6) * kStage;
  int nst = 0;
  for (uint64_t i = wave; i < count; i += nwaves) {
    const int32_t v = qin[i];
    const int64_t e0 = rp[v], e1 = rp[v + 1];
    for (int64_t e = e0; e < e1; e += 64) {
      const int64_t my = e + lane;
      bool enq = false;
      int32_t u = 0;
      if (my < e1) {
        u = col[my];
        const uint32_t bit = 1u << (u & 31);
        if (!(bitmap[u >> 5] & bit)) enq = !(atomicOr(&bitmap[u >> 5], bit) & bit);
        if (enq && lev) lev[u] = (uint8_t)(level + 1 < 254 ? level + 1 : 254);
        if (enq) arcs += (uint64_t)(rp[u + 1] - rp[u]);
      }
      const ull eb = __ballot(enq);
      if (eb != 0ull) {
        const int c = __popcll(eb);
        // every vertex is claimed once, so the queue (length n) cannot overflow
        if (nst + c > kStage) stage_flush(stg, nst, qout_n, (uint32_t *)qout, 0, ~0ull, nullptr);
        if (enq) stg[nst + lanes_below(eb)] = (uint32_t)u;
        nst += c;
      }
    }
  }
  stage_flush(stg, nst, qout_n, (uint32_t *)qout, 0, ~0ull, nullptr);
  wave_add_u64(qout_a, arcs);
}

// The same level bottom-up, for a traversal that only needs the set of
// vertices reached (no levels): every vertex not yet reached scans its arcs
// in the opposite direction (rp / col of the other CSR) and joins as soon as
// one of them leads to a reached vertex.  A vertex reached earlier in the
// same launch may be the one found, which can put a vertex in this level
// that the top-down order would put in a later one; the set is the same.
// Runs only when the frontier has at least bu_arcs arcs to scan top-down.
// One thread per vertex; the vertices that join are appended, with their
// arc counts in the top-down CSR (rp_td), as the top-down kernel appends
// them, so the next level can go either way.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_reach_bu(const int64_t *rp, const int32_t *col, const int64_t *rp_td,
                                                    uint32_t *bitmap, const uint64_t *qin_a, int32_t *qout,
                                                    uint32_t *qout_n, uint64_t *qout_a, int64_t n,
                                                    uint64_t bu_arcs) {
  if (*qin_a < bu_arcs) return;
  uint64_t arcs = 0;
  const uint64_t tid = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
  const uint64_t nth = (uint64_t)gridDim.x * BLOCK;
  __shared__ uint32_t st_all[(BLOCK / 64) * kStage];
  uint32_t *stg = st_all + (threadIdx.x >> 6) * kStage;
  int nst = 0;
  // the loop bound is the same for every lane of a wavefront (whole
  // wavefronts stride together), so the ballots below see every lane
  const uint64_t span = (((uint64_t)n + 63) / 64) * 64;
  for (uint64_t u = tid; u < span; u += nth) {
    bool join = false;
    if (u < (uint64_t)n && !((bitmap[u >> 5] >> (u & 31)) & 1u)) {
      const int64_t e1 = rp[u + 1];
      for (int64_t e = rp[u]; e < e1; ++e) {
        const uint32_t w = (uint32_t)col[e];
        if ((bitmap[w >> 5] >> (w & 31)) & 1u) {
          join = true;
          break;
        }
      }
      if (join) {
        atomicOr(&bitmap[u >> 5], 1u << (u & 31));
        arcs += (uint64_t)(rp_td[u + 1] - rp_td[u]);
      }
    }
    const ull eb = __ballot(join);
    if (eb != 0ull) {
      const int c = __popcll(eb);
      if (nst + c > kStage) stage_flush(stg, nst, qout_n, (uint32_t *)qout, 0, ~0ull, nullptr);
      if (join) stg[nst + lanes_below(eb)] = (uint32_t)u;
      nst += c;
    }
  }
  stage_flush(stg, nst, qout_n, (uint32_t *)qout, 0, ~0ull, nullptr);
  wave_add_u64(qout_a, arcs);
}

// Streaming probes over n16 16-byte words: every thread keeps four 16-byte
// loads in flight (one per grid stride) before it uses them, so the probe is
// bound by HBM and not by the latency of one load at a time.  Copy: loads and
// stores marked non-temporal (streamed past the caches).  Read: the words are
// folded into one value that is stored only if it matches a sentinel, so the
// loads cannot be dropped.
typedef unsigned v4u __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy(const v4u *__restrict__ src, v4u *__restrict__ dst, int64_t n16) {
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * nth < n16; i += 4 * nth) {
    v4u v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(&src[i + u * nth]);
#pragma unroll
    for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], &dst[i + u * nth]);
  }
  for (; i < n16; i += nth) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_read(const v4u *__restrict__ src, int64_t n16, unsigned *sink) {
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned acc = 0;
  for (; i + 3 * nth < n16; i += 4 * nth) {
    v4u v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = src[i + u * nth];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  for (; i < n16; i += nth) acc ^= src[i].x;
  if (acc == 0x9E3779B9u) sink[0] = acc;
}

// ------------------------------------------------------------ launchers

#define DISPATCH_BLOCK(L, KERNEL, ...)                                                     \
  do {                                                                                     \
    switch ((L).block) {                                                                   \
      case 64: hipLaunchKernelGGL(KERNEL<64>, dim3((L).grid), dim3(64), 0, st, __VA_ARGS__); break;    \
      case 128: hipLaunchKernelGGL(KERNEL<128>, dim3((L).grid), dim3(128), 0, st, __VA_ARGS__); break; \
      case 512: hipLaunchKernelGGL(KERNEL<512>, dim3((L).grid), dim3(512), 0, st, __VA_ARGS__); break; \
      default: hipLaunchKernelGGL(KERNEL<256>, dim3((L).grid), dim3(256), 0, st, __VA_ARGS__); break;  \
    }                                                                                      \
  } while (0)

hipError_t launch_batch_init(const BatchState &S, const uint32_t *items0, const ull *masks0, const uint32_t *dest0,
                             int k, hipStream_t st) {
  if (k <= 0) return hipSuccess;
  const int grid = (k + 255) / 256;
  hipLaunchKernelGGL(k_batch_init, dim3(grid), dim3(256), 0, st, S, items0, masks0, dest0, k);
  return hipGetLastError();
}

template <int K>
static void launch_fwd_k(const DevGraph &G, const BatchState &S, int level, const Launch &L, hipStream_t st) {
  if (S.push) {
    switch (L.block) {
      case 64: k_fwd_push<64, K><<<dim3(L.grid), dim3(64), 0, st>>>(G, S, level); break;
      case 128: k_fwd_push<128, K><<<dim3(L.grid), dim3(128), 0, st>>>(G, S, level); break;
      case 512: k_fwd_push<512, K><<<dim3(L.grid), dim3(512), 0, st>>>(G, S, level); break;
      default: k_fwd_push<256, K><<<dim3(L.grid), dim3(256), 0, st>>>(G, S, level); break;
    }
    return;
  }
  switch (L.block) {
    case 64: k_fwd_level<64, K><<<dim3(L.grid), dim3(64), 0, st>>>(G, S, level); break;
    case 128: k_fwd_level<128, K><<<dim3(L.grid), dim3(128), 0, st>>>(G, S, level); break;
    case 512: k_fwd_level<512, K><<<dim3(L.grid), dim3(512), 0, st>>>(G, S, level); break;
    default: k_fwd_level<256, K><<<dim3(L.grid), dim3(256), 0, st>>>(G, S, level); break;
  }
}

template <int K>
static void launch_bu_k(const DevGraph &G, const BatchState &S, int level, const Launch &L, hipStream_t st) {
  switch (L.block) {
    case 64: k_bu_level<64, K><<<dim3(L.grid), dim3(64), 0, st>>>(G, S, level); break;
    case 128: k_bu_level<128, K><<<dim3(L.grid), dim3(128), 0, st>>>(G, S, level); break;
    case 512: k_bu_level<512, K><<<dim3(L.grid), dim3(512), 0, st>>>(G, S, level); break;
    default: k_bu_level<256, K><<<dim3(L.grid), dim3(256), 0, st>>>(G, S, level); break;
  }
}

hipError_t launch_bu_level(const DevGraph &G, const BatchState &S, int level, Launch L, hipStream_t st) {
  switch (L.items) {
    case 2: launch_bu_k<2>(G, S, level, L, st); break;
    case 4: launch_bu_k<4>(G, S, level, L, st); break;
    default: launch_bu_k<1>(G, S, level, L, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_fwd_level(const DevGraph &G, const BatchState &S, int level, Launch L, hipStream_t st) {
  switch (L.items) {
    case 2: launch_fwd_k<2>(G, S, level, L, st); break;
    case 4: launch_fwd_k<4>(G, S, level, L, st); break;
    default: launch_fwd_k<1>(G, S, level, L, st); break;
  }
  return hipGetLastError();
}

template <int K>
static void launch_bwd_k(const DevGraph &G, const BatchState &S, int level, int ntgt, int full, const Launch &L,
                         hipStream_t st) {
  switch (L.block) {
    case 64: k_bwd_level<64, K><<<dim3(L.grid), dim3(64), 0, st>>>(G, S, level, ntgt, full); break;
    case 128: k_bwd_level<128, K><<<dim3(L.grid), dim3(128), 0, st>>>(G, S, level, ntgt, full); break;
    case 512: k_bwd_level<512, K><<<dim3(L.grid), dim3(512), 0, st>>>(G, S, level, ntgt, full); break;
    default: k_bwd_level<256, K><<<dim3(L.grid), dim3(256), 0, st>>>(G, S, level, ntgt, full); break;
  }
}

hipError_t launch_bwd_level(const DevGraph &G, const BatchState &S, int level, int ntgt, int full, Launch L,
                            hipStream_t st) {
  switch (L.items) {
    case 2: launch_bwd_k<2>(G, S, level, ntgt, full, L, st); break;
    case 4: launch_bwd_k<4>(G, S, level, ntgt, full, L, st); break;
    default: launch_bwd_k<1>(G, S, level, ntgt, full, L, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_batch_cleanup(const BatchState &S, const PartTotals &tot, Launch L, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_cleanup, dim3(L.grid), dim3(256), 0, st, S, tot);
  return hipGetLastError();
}

hipError_t launch_batch_export(const BatchState &S, int level, uint64_t begin, uint64_t count,
                               const int32_t *lane_slot, uint64_t *dist, ull *sigma, double *delta, int64_t k,
                               hipStream_t st) {
  if (count == 0) return hipSuccess;
  uint64_t waves = count < 65536 ? count : 65536;
  const int grid = (int)((waves * 64 + 255) / 256);
  hipLaunchKernelGGL(k_batch_export, dim3(grid), dim3(256), 0, st, S, level, begin, count, lane_slot, dist,
                     sigma, delta, k);
  return hipGetLastError();
}

hipError_t launch_plain_init(const PlainState &P, int32_t s, hipStream_t st) {
  hipLaunchKernelGGL(k_plain_init, dim3(1), dim3(64), 0, st, P, s);
  return hipGetLastError();
}

hipError_t launch_plain_fwd(const DevGraph &G, const PlainState &P, int level, Launch L, hipStream_t st) {
  DISPATCH_BLOCK(L, k_plain_fwd, G, P, level);
  return hipGetLastError();
}

hipError_t launch_plain_bwd(const DevGraph &G, const PlainState &P, int level, int32_t target, int only_target,
                            Launch L, hipStream_t st) {
  DISPATCH_BLOCK(L, k_plain_bwd, G, P, level, target, only_target);
  return hipGetLastError();
}

hipError_t launch_plain_cleanup(const PlainState &P, uint64_t total, hipStream_t st) {
  if (total == 0) return hipSuccess;
  uint64_t g = (total + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_plain_cleanup, dim3((int)g), dim3(256), 0, st, P, total);
  return hipGetLastError();
}

hipError_t launch_plain_export(const PlainState &P, uint64_t *dist, ull *sigma, double *delta,
                               hipStream_t st) {
  uint64_t g = ((uint64_t)P.n + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_plain_export, dim3((int)g), dim3(256), 0, st, P, dist, sigma, delta);
  return hipGetLastError();
}

hipError_t launch_plain_export(const PlainState &P, uint64_t total, uint64_t *dist, ull *sigma, double *delta,
                               hipStream_t st) {
  (void)total;
  return launch_plain_export(P, dist, sigma, delta, st);
}

hipError_t launch_reach_init(uint32_t *bitmap, int32_t *q, uint32_t *qn, int32_t root, hipStream_t st) {
  hipLaunchKernelGGL(k_reach_init, dim3(1), dim3(64), 0, st, bitmap, q, qn, root);
  return hipGetLastError();
}

hipError_t launch_reach_level(const int64_t *rp, const int32_t *col, uint32_t *bitmap, const int32_t *qin,
                              const uint32_t *qin_n, const uint64_t *qin_a, int32_t *qout, uint32_t *qout_n,
                              uint64_t *qout_a, uint8_t *lev, int level, uint64_t bu_arcs, Launch L,
                              hipStream_t st) {
  DISPATCH_BLOCK(L, k_reach_level, rp, col, bitmap, qin, qin_n, qin_a, qout, qout_n, qout_a, lev, level, bu_arcs);
  return hipGetLastError();
}

hipError_t launch_reach_bu(const int64_t *rp, const int32_t *col, const int64_t *rp_td, uint32_t *bitmap,
                           const uint64_t *qin_a, int32_t *qout, uint32_t *qout_n, uint64_t *qout_a, int64_t n,
                           uint64_t bu_arcs, Launch L, hipStream_t st) {
  DISPATCH_BLOCK(L, k_reach_bu, rp, col, rp_td, bitmap, qin_a, qout, qout_n, qout_a, n, bu_arcs);
  return hipGetLastError();
}

hipError_t launch_copy_probe(const void *src, void *dst, int64_t n16, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, st, static_cast<const v4u *>(src), static_cast<v4u *>(dst),
                     n16);
  return hipGetLastError();
}

hipError_t launch_read_probe(const void *src, int64_t n16, unsigned *sink, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_read, dim3(grid), dim3(256), 0, st, static_cast<const v4u *>(src), n16, sink);
  return hipGetLastError();
}

// ------------------------------------------------------------- targets

__global__ void k_scatter_targets(int32_t *tgt_of, const int32_t *verts, int k, int set) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x)
    tgt_of[verts[i]] = set ? i : -1;
}

// Plain engine: distance and delta of each listed vertex.
__global__ void k_plain_gather(PlainState P, const int32_t *verts, int k, int32_t *d_out, double *delta_out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    const int32_t v = verts[i];
    if (d_out) d_out[i] = P.d[v];
    if (delta_out) delta_out[i] = P.d[v] < 0 ? 0.0 : P.dout[v];
  }
}

// Adds the per-workgroup counter slots into acc and clears them: a thread
// per slot row (rows are contiguous, so the reads coalesce), a wavefront
// sum per counter, one atomic per counter and wavefront.  Integer sums:
// the order does not matter.
constexpr int kFoldBlock = 256;
__global__ __launch_bounds__(kFoldBlock) void k_ctr_fold(uint64_t *ctr, int slots, uint64_t *acc) {
  uint64_t s[C_COUNT];
#pragma unroll
  for (int k = 0; k < C_COUNT; ++k) s[k] = 0;
  for (int i = blockIdx.x * kFoldBlock + threadIdx.x; i < slots; i += gridDim.x * kFoldBlock) {
    uint64_t *row = ctr + (size_t)i * C_COUNT;
#pragma unroll
    for (int k = 0; k < C_COUNT; ++k) {
      s[k] += row[k];
      row[k] = 0;
    }
  }
#pragma unroll
  for (int k = 0; k < C_COUNT; ++k) {
    uint64_t v = s[k];
    for (int off = 32; off > 0; off >>= 1) v += (uint64_t)__shfl_xor((unsigned long long)v, off);
    if (lane_id() == 0 && v != 0) atomicAdd((unsigned long long *)&acc[k], (unsigned long long)v);
  }
}

hipError_t launch_ctr_fold(uint64_t *ctr, int slots, uint64_t *acc, hipStream_t st) {
  const int grid = std::max(1, std::min(32, (slots + kFoldBlock - 1) / kFoldBlock));
  hipLaunchKernelGGL(k_ctr_fold, dim3(grid), dim3(kFoldBlock), 0, st, ctr, slots, acc);
  return hipGetLastError();
}

__global__ void k_route_results(const double *res, const ResultRoute *routes, int k) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x)
    *routes[i].dst = res[routes[i].src];
}

hipError_t launch_route_results(const double *res, const ResultRoute *routes, int k, hipStream_t st) {
  if (k <= 0) return hipSuccess;
  const int grid = std::min(4096, (k + 255) / 256);
  hipLaunchKernelGGL(k_route_results, dim3(grid), dim3(256), 0, st, res, routes, k);
  return hipGetLastError();
}

hipError_t launch_scatter_targets(int32_t *tgt_of, const int32_t *verts, int k, int set, hipStream_t st) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_targets, dim3((k + 255) / 256), dim3(256), 0, st, tgt_of, verts, k, set);
  return hipGetLastError();
}

hipError_t launch_plain_gather(const PlainState &P, const int32_t *verts, int k, int32_t *d_out,
                               double *delta_out, hipStream_t st) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_plain_gather, dim3((k + 255) / 256), dim3(256), 0, st, P, verts, k, d_out, delta_out);
  return hipGetLastError();
}

}  // namespace bcd
