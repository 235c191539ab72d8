// bitsort_device.h -- wavefront / block primitives for gfx950 (wave64).
//
// Everything here is device code used by the kernels in bitsort.hip.  The
// prefix sums count set bits (Example 6 of Section III of the paper: the
// number of ones in a word) and combine them across lanes with ballot and
// mbcnt, the cross-lane primitives of the CDNA ISA.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace bitsort_dev {

constexpr uint32_t kWave = 64;

// Status block kept at the start of every workspace (layout of
// bitsort_status_t followed by private counters).
struct Status {
  uint32_t flags;   // BITSORT_STATUS_* bits
  uint32_t done;    // kFinishPending while the totals wait for the status read, else 0
  uint64_t count;   // keys written
};

// A two-kernel plain sort whose caller reads its status through the library
// does not launch its one-workgroup finish step: the slice kernel leaves
// Status::done = kFinishPending and, kPendingOffset bytes into the workspace,
// what the finish step needs.  Reading the status then runs that step (totals,
// flags and, only after a repeated key, the compaction of the output) on the
// stream before copying the status out.
constexpr uint32_t kFinishPending = 0x464E5350u;
constexpr uint32_t kPendingOffset = 64;
struct PendingFinish {
  uint64_t n;             // keys given
  const uint64_t* info;   // per-slice (base, ones, keys) triples
  uint32_t* out;          // the sorted output
  uint32_t nb;            // slices
  uint32_t keep;          // status flags raised by the slice kernel that the finish step keeps
};

__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Values read from LDS or memory are per-lane as far as the compiler knows.
// Any such value that decides a branch or loop around a barrier or a
// cross-lane operation goes through uniform() first: it then lives in a
// scalar register and the branch is a scalar one, so every wave takes it the
// same way and executes the same barriers.
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint64_t uniform(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Number of set bits of `m` in lanes below the calling lane.
__device__ __forceinline__ uint32_t count_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

// Exclusive wave prefix of c in [0, 63] built from six ballots (one per bit
// plane of c) and mbcnt; *total receives the wave's sum.
__device__ __forceinline__ uint32_t wave_prefix_small(uint32_t c, uint32_t* total) {
  uint32_t p = 0, t = 0;
#pragma unroll
  for (uint32_t k = 0; k < 6; ++k) {
    const uint64_t m = __ballot((c >> k) & 1u);
    p += count_below(m) << k;
    t += static_cast<uint32_t>(__popcll(m)) << k;
  }
  *total = t;
  return p;
}

// DPP lane moves of a wave64 (four rows of 16 lanes): row_shr:k takes lane
// i - k of the same row (0 past the row's start, bound_ctrl), row_bcast:15
// and row_bcast:31 take lane 15 of the previous row and lane 31 into the
// rows the row mask enables (0 in the others).
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ uint32_t dpp_or_zero(uint32_t v) {
  return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), CTRL, ROW_MASK, 0xf, BOUND));
}

// Inclusive scan of u32 values over the 64 lanes (every lane active): sums
// within each row of 16 by shifts of 1, 2, 4 and 8 lanes, then row 0's total
// into row 1 and row 2's into row 3 (row_bcast:15), then the first two rows'
// total into rows 2 and 3 (row_bcast:31).  Six VALU moves instead of six
// LDS-routed shuffles.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  v += dpp_or_zero<0x111, 0xf, true>(v);  // row_shr:1
  v += dpp_or_zero<0x112, 0xf, true>(v);  // row_shr:2
  v += dpp_or_zero<0x114, 0xf, true>(v);  // row_shr:4
  v += dpp_or_zero<0x118, 0xf, true>(v);  // row_shr:8
  v += dpp_or_zero<0x142, 0xa, false>(v); // row_bcast:15
  v += dpp_or_zero<0x143, 0xc, false>(v); // row_bcast:31
  return v;
}

// Sum of u32 values over the wave (mod 2^32), in a scalar register.
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
  return __builtin_amdgcn_readlane(wave_incl_scan(v), kWave - 1);
}

// Sum of u64 values over the wave (mod 2^64): the low 32 bits in two 16-bit
// halves (each sum stays below 2^22) and the high 32 bits, each summed over
// the lanes in 32 bits.
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
  const uint64_t a = wave_sum_u32(static_cast<uint32_t>(v) & 0xFFFFu);
  const uint64_t b = wave_sum_u32(static_cast<uint32_t>(v) >> 16);
  const uint64_t c = wave_sum_u32(static_cast<uint32_t>(v >> 32));
  return a + (b << 16) + (c << 32);
}

// Exclusive block scan of one u32 per thread.  `scratch` holds BLOCK/64
// words of LDS.  Contains two barriers; every thread must call it.
template <int BLOCK>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* scratch, uint32_t* total) {
  constexpr uint32_t kWaves = BLOCK / kWave;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t wave = threadIdx.x / kWave;
  const uint32_t inc = wave_incl_scan(v);
  if (lane == kWave - 1) scratch[wave] = inc;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (uint32_t i = 0; i < kWaves; ++i) {
    const uint32_t s = scratch[i];
    base += (i < wave) ? s : 0u;
    tot += s;
  }
  __syncthreads();
  *total = uniform(tot);
  return base + inc - v;
}

// Block sum of one u64 per thread; `scratch` holds BLOCK/64 u64 of LDS.
template <int BLOCK>
__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t* scratch) {
  constexpr uint32_t kWaves = BLOCK / kWave;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t wave = threadIdx.x / kWave;
  v = wave_sum_u64(v);
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  uint64_t tot = 0;
#pragma unroll
  for (uint32_t i = 0; i < kWaves; ++i) tot += scratch[i];
  __syncthreads();
  return uniform(tot);
}

// A pointer known to address device memory, such as one read from a
// descriptor in memory: the cast lets the compiler use global instead of flat
// loads and stores through it (a flat access also waits on the LDS counter).
template <typename T>
__device__ __forceinline__ T* as_global(T* p) {
  return (T*)((__attribute__((address_space(1))) T*)reinterpret_cast<uintptr_t>(p));
}

__device__ __forceinline__ uint32_t atomic_load_flags(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace bitsort_dev
