// Device helpers shared by the kernel files of libbcd (wave64 primitives
// and per-workgroup counter flushing).
#pragma once

#include "bcd_internal.h"

namespace bcd {

typedef unsigned long long ull;

static __device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

static __device__ __forceinline__ int lanes_below(ull m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

static __device__ __forceinline__ uint32_t read_lane(uint32_t x, int j) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, j);
}

static __device__ __forceinline__ ull read_lane64(ull x, int j) {
  uint32_t lo = read_lane((uint32_t)x, j);
  uint32_t hi = read_lane((uint32_t)(x >> 32), j);
  return ((ull)hi << 32) | lo;
}

static __device__ __forceinline__ uint64_t first_lane64(uint64_t x) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Sum three per-thread counters over the workgroup and add them into this
// workgroup's private counter slot (one writer per slot per launch).
template <int BLOCK>
__device__ __forceinline__ void flush_counters(uint64_t *ctr, int slots, int k0, uint64_t a, uint64_t b,
                                               uint64_t c, bool ovf, uint32_t *flags) {
  __shared__ uint64_t red[3][BLOCK / 64];
  __shared__ int any_ovf;
  if (threadIdx.x == 0) any_ovf = 0;
  __syncthreads();
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off);
    b += __shfl_down(b, off);
    c += __shfl_down(c, off);
  }
  if (ovf) any_ovf = 1;
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) {
    red[0][w] = a;
    red[1][w] = b;
    red[2][w] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t s0 = 0, s1 = 0, s2 = 0;
    for (int i = 0; i < BLOCK / 64; ++i) {
      s0 += red[0][i];
      s1 += red[1][i];
      s2 += red[2][i];
    }
    if ((int)blockIdx.x < slots) {
      uint64_t *p = ctr + (size_t)blockIdx.x * C_COUNT + k0;
      p[0] += s0;
      p[1] += s1;
      p[2] += s2;
    }
    if (any_ovf) atomicOr(&flags[0], 1u);
  }
}

// Add wave-uniform counters (the same value on every lane of a wavefront)
// into this workgroup's slot: counter slot k[i] receives the sum over the
// workgroup's wavefronts of v[i]; an overflow on any lane raises flags[0].
// Every thread of the workgroup must call it (once per launch).
template <int BLOCK, int NV>
__device__ __forceinline__ void flush_wave_counters(uint64_t *ctr, int slots, const int (&k)[NV],
                                                    const uint64_t (&v)[NV], bool ovf, uint32_t *flags) {
  __shared__ uint64_t red[NV][BLOCK / 64];
  __shared__ int any_ovf;
  if (threadIdx.x == 0) any_ovf = 0;
  __syncthreads();
  if (ovf) any_ovf = 1;
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0)
    for (int i = 0; i < NV; ++i) red[i][w] = v[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    if ((int)blockIdx.x < slots) {
      uint64_t *p = ctr + (size_t)blockIdx.x * C_COUNT;
      for (int i = 0; i < NV; ++i) {
        uint64_t s = 0;
        for (int j = 0; j < BLOCK / 64; ++j) s += red[i][j];
        p[k[i]] += s;
      }
    }
    if (any_ovf) atomicOr(&flags[0], 1u);
  }
}

// Per-wavefront LDS staging of list appends: values are collected in an LDS
// buffer and copied out with one tail atomic per block, so a list's shared
// tail counter is not hit once per appended element.
static __device__ __forceinline__ void stage_flush(uint32_t *buf, int &nbuf, uint32_t *tail, uint32_t *dst,
                                                   uint64_t dst_base, uint64_t dst_end, uint32_t *overflow_flag) {
  if (nbuf == 0) return;
  uint32_t p0 = 0;
  if ((threadIdx.x & 63) == 0) p0 = atomicAdd(tail, (uint32_t)nbuf);
  p0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)p0);
  for (int j = (int)(threadIdx.x & 63); j < nbuf; j += 64) {
    const uint64_t p = dst_base + p0 + (uint64_t)j;
    if (p < dst_end) dst[p] = buf[j];
    else if (overflow_flag) atomicOr(overflow_flag, 1u);
  }
  nbuf = 0;
}

// Append one wave-uniform value (when `pred` is true on the wavefront).
template <int CAP>
static __device__ __forceinline__ void stage_one(uint32_t *buf, int &nbuf, bool pred, uint32_t value, uint32_t *tail,
                                                 uint32_t *dst, uint64_t dst_base, uint64_t dst_end,
                                                 uint32_t *overflow_flag) {
  if (!pred) return;
  if (nbuf == CAP) stage_flush(buf, nbuf, tail, dst, dst_base, dst_end, overflow_flag);
  if ((threadIdx.x & 63) == 0) buf[nbuf] = value;
  nbuf += 1;
}

// Append the value of every lane where `pred` holds (lane order kept).
template <int CAP>
static __device__ __forceinline__ void stage_lanes(uint32_t *buf, int &nbuf, bool pred, uint32_t value, uint32_t *tail,
                                                   uint32_t *dst, uint64_t dst_base, uint64_t dst_end,
                                                   uint32_t *overflow_flag) {
  const ull m = __ballot(pred);
  if (m == 0ull) return;
  const int c = __popcll(m);
  if (nbuf + c > CAP) stage_flush(buf, nbuf, tail, dst, dst_base, dst_end, overflow_flag);
  if (pred) buf[nbuf + lanes_below(m)] = value;
  nbuf += c;
}

// This workgroup's share of a partitioned item list (see BatchState).
struct PartView {
  int p;              // partition served
  uint64_t wave;      // this wavefront's index within the partition
  uint64_t nwaves;    // wavefronts serving the partition
  uint64_t thread;    // this thread's index within the partition
  uint64_t nthreads;
};

template <int BLOCK>
static __device__ __forceinline__ PartView part_view(int P) {
  PartView r;
  r.p = (int)(blockIdx.x % (unsigned)P);
  const uint64_t lb = blockIdx.x / (unsigned)P, nwg = gridDim.x / (unsigned)P;
  r.wave = (lb * BLOCK + threadIdx.x) >> 6;
  r.nwaves = (nwg * BLOCK) >> 6;
  r.thread = lb * BLOCK + threadIdx.x;
  r.nthreads = nwg * BLOCK;
  return r;
}

}  // namespace bcd
