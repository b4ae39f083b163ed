// Internal declarations shared by the host layer and the HIP kernels of
// libbcd.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bcd {

constexpr int kLanes = 64;  // sources per column group = wavefront width on gfx950

// Entry of the backward pass's level-tagged mask table: which lanes of a
// vertex sit on level `lev` of batch `epoch`.
struct __align__(16) LevMask {
  unsigned long long mask;
  uint32_t lev;
  uint32_t epoch;
};

// All level masks of one (group, vertex) of the unweighted engine in one
// 64-byte record, so the test "is w settled for these sources" and the flag
// for the next level touch a single cache line per arc.
struct __align__(64) MaskRec {
  unsigned long long vis;    // lanes settled on a level < current (lagging, see the forward kernel)
  unsigned long long fr[4];  // rotating level masks: current, next, previous, retiring
  unsigned long long dn;     // lanes on whose shortest-path DAG the vertex is a target or lies below one
  unsigned long long pad[2];
};

// Counters accumulated per workgroup slot (no atomics), reduced on the host.
enum Ctr {
  C_FWD_VPAIRS = 0,  // (source, vertex) pairs expanded by the forward kernel
  C_FWD_APAIRS = 1,  // (source, arc) pairs scanned by the forward kernel  (= sum m_s)
  C_FWD_DPAIRS = 2,  // (source, DAG arc) pairs the forward kernel pushed sigma along (= sum a_s)
  C_BWD_VPAIRS = 3,  // (source, vertex) pairs whose psi the backward kernel produced
  C_BWD_APAIRS = 4,  // (source, arc) pairs the backward kernel scanned
  C_BWD_DPAIRS = 5,  // (source, DAG arc) pairs the backward kernel accumulated
  C_RLX_APAIRS = 6,  // (source, arc) relaxations of the weighted distance rounds (6..8)
  C_SCRATCH = 9,     // unused slots for kernels that only report overflow (9..11)
  C_FWD_ITEMS = 12,  // work items (64-source group, vertex, level) of the forward
  C_FWD_IARCS = 13,  // sum over those items of the vertex's out-degree
  C_BWD_ITEMS = 14,  // work items the backward computed psi for
  C_BWD_IARCS = 15,  // sum over those items of the vertex's out-degree
  C_COUNT = 16
};

// Device state of one batch of G column groups (64 sources each) over an
// n-vertex graph.  All [G][n][64] arrays are vertex-major inside a group, so
// the 64 sources of one vertex are one contiguous row a wavefront reads or
// writes with one coalesced access.
struct BatchState {
  int64_t n;
  int G;
  unsigned long long *sig;   // [G][n][64] path counts
  double *psi;               // [G][n][64] (1 + delta) / sigma
  double *dout;              // [G][n][64] delta, verification hook only (may be null)
  MaskRec *rec;              // [G][n] level masks (unweighted engine)
  unsigned long long *vis;   // [G][n] reached lanes (weighted engine)
  unsigned long long *fr;    // [3][G][n] rotating round masks (weighted engine)
  LevMask *bt;               // [2][G][n] backward level masks, by level parity
  // Item lists are split into P partitions (group g belongs to partition
  // g % P); workgroup b serves partition b % P, so with P = 8 every XCD
  // (workgroups are dealt to the 8 XCDs round-robin) walks only its own
  // groups and their masks stay in that XCD's L2.  Partition p owns items
  // [p * capP, (p + 1) * capP).
  uint32_t *items;           // [cap] g * n + v, grouped by partition, then level
  unsigned long long *imask; // [cap] lanes of the item on its level
  uint64_t cap;              // = P * capP
  uint64_t capP;
  int P;
  uint32_t *cnt;             // [(n + 2) * 8] items per (level, partition): index level * P + p
  uint64_t *off;             // [(n + 2) * 8] first item of each (level, partition)
  uint32_t *tmin;            // [1] smallest over all lanes
  int32_t *tgt_of;           // [n] target index of a vertex, -1 if none
  double *res;               // [ntgt][G][64] delta of lane on target
  uint64_t *ctr;             // [grid][C_COUNT] per-workgroup counters
  uint64_t *acc;             // [C_COUNT] counters of completed batches
  uint32_t *flags;           // [4]: 0 sigma overflow, 1 item capacity exceeded
  unsigned long long *ovl;   // [G] lanes whose sigma overflowed
  uint32_t epoch;
  int ctr_slots;
  // per batch (unweighted engine)
  int gused;                     // column groups holding sources: 0 .. gused-1
  unsigned long long last_lanes; // lanes of group gused-1 that hold a source
  int bu_den;                    // bottom-up levels: see level_bottom_up (0 = never)
  int keep_all;                  // 1: the backward runs on every lane (exports), else only below a target
  int push;                      // 1: top-down levels push path counts along DAG arcs (k_fwd_push), 0: pull
  // weighted graphs only
  uint32_t *wd;              // [G][n][64] distances, 0xFFFFFFFF unreached
  uint32_t *wc;              // [G][n][64] shortest-path-DAG in-arcs not yet pushed
  unsigned long long *chg;   // [2][G][n] lanes whose distance dropped (relaxation rounds)
  uint32_t *bq;              // [2][G*n] relaxation round queues
  uint32_t *bqn;             // [3] relaxation queue lengths (rotating)
  uint32_t *rl;              // [G*n] items reached by any lane
  uint32_t *rln;             // [1]
  unsigned long long *wdn;   // [G][n] lanes on whose DAG the vertex is a target or lies below one
  unsigned long long *dagm;  // [G][m] lanes on whose shortest-path DAG the arc lies, by transpose position
};

// Plain engine state (one source).
struct PlainState {
  int64_t n;
  int32_t *d;                // [n] level, -1 unreached
  unsigned long long *sig;   // [n]
  double *psi;               // [n]
  double *dout;              // [n] delta, verification only
  int32_t *queue;            // [n] vertices by level
  uint32_t *cnt;             // [n + 2]
  uint64_t *off;             // [n + 2]
  uint64_t *ctr;             // [grid][C_COUNT]
  uint64_t *acc;             // [C_COUNT]
  uint32_t *flags;           // [4]
  int ctr_slots;
};

struct DevGraph {
  int64_t n, m;
  const int64_t *rp;    // [n+1]
  const int32_t *col;   // [m]
  const int64_t *irp;   // transpose
  const int32_t *icol;
  // weighted graphs: arc fields in pairs, so that one 8-byte load brings what
  // a kernel reads of an arc (separate 4-byte arrays and one 16-byte record
  // of all fields both measured slower)
  const uint2 *arcw;    // [m] CSR order: {head, length} (relaxation)
  const uint2 *arcp;    // [m] CSR order: {head, position of the arc in the transpose} (sigma, backward)
  const uint2 *iarc;    // [m] transpose order: {tail, length} (DAG in-degrees)
};

// Whether BFS level `level` (>= 2) of a batch is found bottom-up, from the
// item count of level-1 (complete before any kernel of `level` starts):
// when level-1 holds at least 1 / bu_den of the batch's (group, vertex)
// pairs, scanning the in-arcs of the unsettled pairs is cheaper than the
// out-arcs of the frontier.  Host and device evaluate the same integer rule.
__host__ __device__ inline bool bottom_up_rule(int bu_den, int level, uint64_t prev_count, int gused, int64_t n) {
  return bu_den > 0 && level >= 2 && prev_count * (uint64_t)bu_den >= (uint64_t)gused * (uint64_t)n;
}

struct Launch {
  int block;      // threads per workgroup
  int grid;       // workgroups
  int items = 1;  // frontier items per wavefront step (unweighted forward)
};

// ---- launchers (bcd_kernels.hip) ----
struct PartTotals {
  uint64_t t[8];  // items per partition over all levels of a batch
};
hipError_t launch_batch_init(const BatchState &S, const uint32_t *items0, const unsigned long long *masks0,
                             const uint32_t *dest0, int k, hipStream_t st);
hipError_t launch_fwd_level(const DevGraph &G, const BatchState &S, int level, Launch L, hipStream_t st);
hipError_t launch_bu_level(const DevGraph &G, const BatchState &S, int level, Launch L, hipStream_t st);
hipError_t launch_bwd_level(const DevGraph &G, const BatchState &S, int level, int ntgt, int full,
                            Launch L, hipStream_t st);
hipError_t launch_batch_cleanup(const BatchState &S, const PartTotals &tot, Launch L, hipStream_t st);
hipError_t launch_batch_export(const BatchState &S, int level, uint64_t begin, uint64_t count,
                               const int32_t *lane_slot, uint64_t *dist, unsigned long long *sigma,
                               double *delta, int64_t k, hipStream_t st);

hipError_t launch_plain_init(const PlainState &P, int32_t s, hipStream_t st);
hipError_t launch_plain_fwd(const DevGraph &G, const PlainState &P, int level, Launch L, hipStream_t st);
hipError_t launch_plain_bwd(const DevGraph &G, const PlainState &P, int level, int32_t target, int full,
                            Launch L, hipStream_t st);
hipError_t launch_plain_cleanup(const PlainState &P, uint64_t total, hipStream_t st);
hipError_t launch_plain_export(const PlainState &P, uint64_t total, uint64_t *dist,
                               unsigned long long *sigma, double *delta, hipStream_t st);

// Reachability BFS over one CSR (reverse graph for RV, forward for FR).
hipError_t launch_reach_init(uint32_t *bitmap, int32_t *q, uint32_t *qn, int32_t root, hipStream_t st);
// Reachability levels: queue lengths *_n and the arcs their vertices have
// in the traversed CSR *_a; a level goes bottom-up (launch_reach_bu, over the
// other CSR) when its frontier has at least bu_arcs arcs, else top-down.
hipError_t launch_reach_level(const int64_t *rp, const int32_t *col, uint32_t *bitmap, const int32_t *qin,
                              const uint32_t *qin_n, const uint64_t *qin_a, int32_t *qout, uint32_t *qout_n,
                              uint64_t *qout_a, uint8_t *lev, int level, uint64_t bu_arcs, Launch L,
                              hipStream_t st);
hipError_t launch_reach_bu(const int64_t *rp, const int32_t *col, const int64_t *rp_td, uint32_t *bitmap,
                           const uint64_t *qin_a, int32_t *qout, uint32_t *qout_n, uint64_t *qout_a, int64_t n,
                           uint64_t bu_arcs, Launch L, hipStream_t st);
hipError_t launch_scatter_targets(int32_t *tgt_of, const int32_t *verts, int k, int set, hipStream_t st);
hipError_t launch_plain_gather(const PlainState &P, const int32_t *verts, int k, int32_t *d_out,
                               double *delta_out, hipStream_t st);
// weighted engine (bcd_weighted.hip)
hipError_t launch_w_init(const BatchState &S, const uint32_t *items0, const unsigned long long *masks0,
                         const uint32_t *dest0, int k, hipStream_t st);
hipError_t launch_w_relax(const DevGraph &G, const BatchState &S, int round, Launch L, hipStream_t st);
hipError_t launch_w_count(const DevGraph &G, const BatchState &S, Launch L, hipStream_t st);
hipError_t launch_w_sigma(const DevGraph &G, const BatchState &S, int round, Launch L, hipStream_t st);
hipError_t launch_w_bwd(const DevGraph &G, const BatchState &S, int round, int ntgt, int full, Launch L,
                        hipStream_t st);
hipError_t launch_w_cleanup(const BatchState &S, Launch L, hipStream_t st);
hipError_t launch_w_export(const BatchState &S, const int32_t *lane_slot, uint64_t *dist,
                           unsigned long long *sigma, double *delta, int64_t k, Launch L, hipStream_t st);
struct ResultRoute {
  double *dst;      // device address in a query's result buffer
  uint32_t src;     // index into res ([ntgt][G][64])
  uint32_t pad;
};
hipError_t launch_route_results(const double *res, const ResultRoute *routes, int k, hipStream_t st);
// Add the per-workgroup counter slots into acc[C_COUNT] and zero them (one
// launch after every completed batch; an aborted batch just zeroes them).
hipError_t launch_ctr_fold(uint64_t *ctr, int slots, uint64_t *acc, hipStream_t st);
hipError_t launch_copy_probe(const void *src, void *dst, int64_t n16, int grid, hipStream_t st);
hipError_t launch_read_probe(const void *src, int64_t n16, unsigned *sink, int grid, hipStream_t st);

}  // namespace bcd
