// RV(r) without allocation, for callers that cannot allocate device or
// pinned host memory (code under HIP graph capture, serving loops and
// harnesses that forbid it).  Same result as bcd_rv: the vertices that reach
// r (Def.1), found by a breadth-first traversal from r on the resident
// reverse graph (Def.3, Prop.2), ascending, r left out.
//
// The traversal's working memory -- the visited bitmap, the two frontier
// queues and their counters -- lives in `scratch`, one file-scope device
// array of kScratchBytes per device, which the GPU holds from module load
// until the process ends.  Host code never passes the array's name to a
// kernel (on the host it names a shadow variable, not device memory): the
// device address of each GPU's copy is looked up once per device with
// hipGetSymbolAddress and kept.  Calls are serialized by a process-wide lock,
// so calls from several host threads do not overlap on the array; every call
// clears the bitmap and counters it uses with a fill kernel before the
// traversal, so nothing of an earlier call survives into its result.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/bcd.h"
#include "bcd_host_internal.h"

namespace bcd {

// Largest graph the scratch holds: 2^22 vertices (R-MAT scale 22).
constexpr int64_t kNoAllocMaxN = int64_t(1) << 22;
constexpr size_t kCtrBytes = 256;  // counters: queue sizes [2], list size, queue arc counts (uint64) at words 4-7
constexpr size_t kBitmapBytes = (size_t)(kNoAllocMaxN / 32) * 4;  // visited bits
constexpr size_t kQueueBytes = (size_t)kNoAllocMaxN * 4;          // one frontier queue (int32 ids)
constexpr size_t kScratchBytes = kCtrBytes + kBitmapBytes + 2 * kQueueBytes;  // 34,079,000 bytes

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;                         // one call at a time in this process
unsigned char *g_scratch_dev[kMaxDevices] = {};  // device address of `scratch` per device

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// One workgroup: the ids of the set bits of bitmap[0 .. words) below n,
// except `skip`, in ascending order into out[]; their number into *count.
// Chunks of 1024 words: a word per thread, an exclusive prefix sum of the
// bit counts over the workgroup (in-wavefront shuffles, then the wavefront
// totals), then each thread writes its word's ids at its offset.
constexpr int kCompactBlock = 1024;

__global__ __launch_bounds__(kCompactBlock) void k_bitmap_compact(const uint32_t *bitmap, int64_t words, int64_t n,
                                                                  int32_t skip, int32_t *out, uint32_t *count) {
  __shared__ uint32_t wave_total[kCompactBlock / 64];
  __shared__ uint32_t base;
  const int lane = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int64_t w0 = 0; w0 < words; w0 += kCompactBlock) {
    const int64_t w = w0 + threadIdx.x;
    uint32_t bits = 0;
    if (w < words) {
      bits = bitmap[w];
      if ((int64_t)(skip >> 5) == w) bits &= ~(1u << (skip & 31));
      const int64_t valid = n - w * 32;
      if (valid < 32) bits &= valid <= 0 ? 0u : ((1u << valid) - 1u);
    }
    const uint32_t c = (uint32_t)__popc(bits);
    uint32_t x = c;  // inclusive prefix sum within the wavefront
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)x, off);
      if (lane >= off) x += y;
    }
    if (lane == 63) wave_total[wv] = x;
    __syncthreads();
    uint32_t before = 0;
    for (int i = 0; i < wv; ++i) before += wave_total[i];
    uint32_t p = base + before + x - c;
    while (bits) {
      const int b = __ffs((int)bits) - 1;
      bits &= bits - 1u;
      out[p++] = (int32_t)(w * 32 + b);
    }
    __syncthreads();  // every thread has read base and wave_total
    if (threadIdx.x == kCompactBlock - 1) base += before + x;
    __syncthreads();
  }
  if (threadIdx.x == 0) *count = base;
}

// Device address of this device's copy of `scratch` (looked up on the first
// call on the device, with that device current).
bcd_status scratch_address(unsigned char **ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return fail_static(BCD_ERR_DEVICE, "no current HIP device");
  }
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail_static(BCD_ERR_DEVICE, "hipGetSymbolAddress of the RV scratch array failed");
    }
    g_scratch_dev[dev] = static_cast<unsigned char *>(p);
  }
  *ptr = g_scratch_dev[dev];
  return BCD_OK;
}

}  // namespace

}  // namespace bcd

using namespace bcd;

#define NA_HIPCHK(expr, msg)                          \
  do {                                                \
    if ((expr) != hipSuccess) {                       \
      (void)hipGetLastError();                        \
      return fail_static(BCD_ERR_DEVICE, msg);        \
    }                                                 \
  } while (0)

extern "C" bcd_status bcd_rv_noalloc(const bcd_graph *gh, bcd_vid r, bcd_vid *out, int64_t cap, int64_t *count) {
  if (!gh || !count) return fail_static(BCD_ERR_INVALID_ARG, "NULL argument");
  const Graph *g = reinterpret_cast<const Graph *>(gh);
  const int64_t n = g->n;
  if (r < 0 || r >= n) return fail_static(BCD_ERR_INVALID_ARG, "r out of range");
  if (n > kNoAllocMaxN) return fail_static(BCD_ERR_UNSUPPORTED, "graph has more vertices than the RV scratch holds (2^22)");
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  unsigned char *base = nullptr;
  bcd_status st0 = scratch_address(&base);
  if (st0 != BCD_OK) return st0;
  uint32_t *ctr = reinterpret_cast<uint32_t *>(base);            // [0], [1]: queue sizes; [2]: list size
  uint32_t *bitmap = reinterpret_cast<uint32_t *>(base + kCtrBytes);
  int32_t *q0 = reinterpret_cast<int32_t *>(base + kCtrBytes + kBitmapBytes);
  int32_t *q1 = reinterpret_cast<int32_t *>(base + kCtrBytes + kBitmapBytes + kQueueBytes);
  const int64_t words = (n + 31) / 32;
  hipStream_t st = nullptr;  // the null stream: every step below is ordered after the one before
  // clear what this call reads before writing it: the bitmap and the counters
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<int64_t>((words + 255) / 256, 1024)), dim3(256), 0, st,
                     bitmap, words, 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, ctr, (int64_t)(kCtrBytes / 4), 0u);
  NA_HIPCHK(hipGetLastError(), "fill launch failed");
  const int64_t *rp = g->d_irp;
  const int32_t *col = g->d_icol;
  if (lds_reach_fits(g)) {
    // small graph: the whole traversal in one workgroup (visited bits and
    // queue in LDS), bitmap written out at the end
    NA_HIPCHK(launch_lds_reach(g, rp, col, r, bitmap, st), "reachability launch failed");
  } else {
    NA_HIPCHK(launch_reach_init(bitmap, q0, &ctr[0], r, st), "reachability launch failed");
    const Launch L = g->launch();
    int32_t *q[2] = {q0, q1};
    int cur = 0;
    // large levels bottom-up over the out-arcs, as the allocating call does;
    // the arcs of queue c's vertices (uint64) at ctr[4 + 2c]
    const uint64_t bu_arcs = (uint64_t)std::max<int64_t>(64, g->m / 64);
    uint64_t *arcs = reinterpret_cast<uint64_t *>(ctr + 4);
    for (int64_t level = 0; level <= n;) {
      // levels 8 at a time between host checks of the frontier size
      for (int i = 0; i < 8; ++i, ++level) {
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, &ctr[1 - cur], (int64_t)1, 0u);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, ctr + 4 + 2 * (1 - cur), (int64_t)2, 0u);
        NA_HIPCHK(hipGetLastError(), "fill launch failed");
        NA_HIPCHK(launch_reach_level(rp, col, bitmap, q[cur], &ctr[cur], &arcs[cur], q[1 - cur], &ctr[1 - cur],
                                     &arcs[1 - cur], nullptr, (int)level, bu_arcs, L, st),
                  "reachability launch failed");
        NA_HIPCHK(launch_reach_bu(g->d_rp, g->d_col, rp, bitmap, &arcs[cur], q[1 - cur], &ctr[1 - cur], &arcs[1 - cur],
                                  n, bu_arcs, L, st),
                  "reachability launch failed");
        cur = 1 - cur;
      }
      uint32_t left = 0;
      NA_HIPCHK(hipMemcpy(&left, &ctr[cur], sizeof(uint32_t), hipMemcpyDeviceToHost), "frontier size copy failed");
      if (left == 0) break;
    }
  }
  // RV(r) ascending into the first queue (free again), its size into ctr[2]
  hipLaunchKernelGGL(k_bitmap_compact, dim3(1), dim3(kCompactBlock), 0, st, bitmap, words, n, (int32_t)r, q0,
                     &ctr[2]);
  NA_HIPCHK(hipGetLastError(), "compaction launch failed");
  uint32_t k = 0;
  NA_HIPCHK(hipMemcpy(&k, &ctr[2], sizeof(uint32_t), hipMemcpyDeviceToHost), "count copy failed");
  *count = (int64_t)k;
  if (!out) return BCD_OK;
  if ((int64_t)k > cap) return fail_static(BCD_ERR_BUFFER_TOO_SMALL, "out holds fewer than |RV(r)| ids");
  if (k > 0) NA_HIPCHK(hipMemcpy(out, q0, (size_t)k * sizeof(int32_t), hipMemcpyDeviceToHost), "RV copy failed");
  return BCD_OK;
}
