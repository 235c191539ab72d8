// bitsort.hip -- host side and C ABI of the gfx950 (MI355X) bitmap sort.
//
// The operation is the one of Yordzhev, arXiv:1312.0138: sort an integer
// array ascending (Section IV, Theorem 1), done here the bit-vector way from
// the primitives of Sections II-III: a key k is marked as bit (k & 31) of
// word (k >> 5) with a shift and an OR (Table I, Examples 2 and 3); the words
// are scanned in order, their ones counted (Example 6), and the position of
// every set bit is written out, lowest bit first (Example 1; bit 0 is the
// rightmost, Section II).
//
// MI355X design.  Global atomics on this part resolve at about 27 G ops/s no
// matter the footprint, so marking n random keys straight into an HBM
// bit-vector costs n atomics at that rate -- tens of times the streaming
// time of the keys.  LDS atomics run at about 2-3 T ops/s.  So keys are never
// marked in HBM: the bit-vector is cut into slices of 2^sb bits that fit in
// one workgroup's LDS (up to 2^20 bits = 128 KiB of the 160 KiB), and the
// keys are routed to their slice first (plain_kernels.inc):
//
//   k_partition  one workgroup per tile of T keys: counts keys per slice
//                (LDS histogram), exclusive-scans the counts, groups the tile
//                by slice in LDS and writes it back coalesced to a staging
//                area at the tile's own offset, plus the tile's per-slice
//                start offsets (a row of the tile table).
//   k_slice      one workgroup per slice: clears its LDS slice, reads that
//                slice's part of every tile (64 keys per wave load, many
//                loads in flight per wave) and ORs the bits in with ds_or.
//                For sparse keys (R/8 > 2n) it then counts ones per word,
//                prefix-sums them with ballot / mbcnt and writes each word's
//                set-bit positions (ctz, clear lowest bit) through LDS so
//                that stores to `out` are contiguous; the slice's output
//                base -- the exclusive prefix over slices -- is the sum over
//                tiles of the tile-local starts.  When the bit-vector is
//                small next to the keys (R/8 <= 2n) it instead writes the
//                slice's words to an HBM bit-vector plus per-chunk prefix
//                counts, and
//   k_emit       scans that bit-vector in 1024-word chunks and writes the
//                keys: many small workgroups share the emission evenly
//                instead of one workgroup per slice.
//   k_finish     one workgroup: totals, status flags, and (only when keys
//                repeat) compaction of the slices' outputs.
//   k_direct     a single workgroup for key ranges that fit one slice and
//                small n: mark, scan and emit without the partition.
//
// HBM traffic of the path: 4n (keys) + 4n + 4n (staging write and read) +
// 4n (out) bytes plus the tile table; the bit-vector adds 2 x R/8 only on the
// k_emit path.  Other files: batch_kernels.inc (segmented batch launch),
// generate.inc (input generator), serve.inc (serving loop).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <vector>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <deque>
#include <functional>
#include <limits>
#include <string>
#include <thread>

#include "bitsort.h"
#include "bitsort_device.h"

using namespace bitsort_dev;

namespace {

#include "plain_kernels.inc"

// ---------------------------------------------------------------------------
#include "generate.inc"

// ---------------------------------------------------------------------------
#include "batch_kernels.inc"

// ---------------------------------------------------------------------------
#include "radix_kernels.inc"

// ---------------------------------------------------------------------------
#include "count_kernels.inc"

// ---------------------------------------------------------------------------
#include "multi_kernels.inc"

// ---------------------------------------------------------------------------
#include "atomic_kernels.inc"

// ---------------------------------------------------------------------------
#include "wide_kernels.inc"

// ---------------------------------------------------------------------------
#include "pairs_kernels.inc"

// ---------------------------------------------------------------------------
// Host side.

struct Plan {
  uint32_t rb = 0, sb = 0, nb = 1, tile_log2 = 0, tile_keys = 0, nt = 0;
  bool direct = true;
  bool via_bitvec = false;  // k_slice writes the bit-vector to HBM, k_emit writes the keys
  bool sparse = false;      // k_slice keeps a summary bit per word and emits only nonzero words
  bool short_units = false; // segments of a few keys: k_slice gathers 16-key units, four per load
  uint64_t n_chunks = 0;
  bool split = false;       // bit-vector route: heavy slices are shared out (k_slice_split)
  size_t off_binfo = 0, off_table = 0, off_staging = 0, off_bitvec = 0, off_chunk = 0, bytes = 0;
  size_t off_split_ctl = 0, off_partials = 0;
  uint32_t stage_cap = 0;
  size_t slice_lds = 0;
  uint32_t bias = 0;  // signed keys: added on load, subtracted on output (mod 2^32)
};

std::atomic<uint32_t> g_tune_sb{0};
std::atomic<uint32_t> g_tune_tile{0};
std::atomic<uint32_t> g_tune_path{0};  // 0 auto, 1 emit from LDS, 2 through the HBM bit-vector
std::mutex g_tune_mu;                   // guards the autotuned tables

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

uint32_t stage_cap_for(uint32_t sb) {
  const uint32_t slice_words = sb >= 5 ? (1u << (sb - 5)) : 1u;
  const uint32_t used = kHeaderBytes + round_up4(slice_words) * 4u;
  uint32_t cap = (kLdsBytes - used) / 4u;
  cap = std::min(cap, kStageMax);
  return cap & ~3u;
}

size_t slice_lds_bytes(uint32_t sb, uint32_t stage_cap) {
  const uint32_t slice_words = sb >= 5 ? (1u << (sb - 5)) : 1u;
  return kHeaderBytes + round_up4(slice_words) * 4u + static_cast<size_t>(stage_cap) * 4u;
}

// Plain-path settings chosen by bitsort_autotune_u32 (or loaded from a
// tuning cache), per (range_bits, ceil(log2 n)).
struct PlainTuning {
  uint32_t slice_bits = 0, tile_log2 = 0, emit_path = 0;
  float ms = 0.f;
};
std::map<std::pair<uint32_t, uint32_t>, PlainTuning> g_plain_tuned;  // guarded by g_tune_mu

uint32_t ceil_log2(uint64_t n) {
  uint32_t l = 0;
  while ((1ull << l) < n) ++l;
  return l;
}

// force != nullptr: use exactly these settings (autotuner candidates),
// ignoring the explicit knobs and the tuned table.
void make_plan(uint64_t n, uint32_t rb, Plan* p, const PlainTuning* force = nullptr) {
  *p = Plan();
  p->rb = rb;
  PlainTuning tuned;
  if (force != nullptr) {
    tuned = *force;
  } else {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_plain_tuned.find({rb, ceil_log2(n)});
    if (it != g_plain_tuned.end()) tuned = it->second;
  }
  if (rb <= kMinSliceBits || (rb <= kMaxSliceBits && n <= kDirectMaxN)) {
    p->direct = true;
    p->sb = rb;
    p->nb = 1;
    p->bytes = kHeaderBytes;
  } else {
    p->direct = false;
    uint32_t sb = force ? 0u : g_tune_sb.load();
    if (sb == 0) sb = tuned.slice_bits;
    if (sb == 0) sb = rb > 8 ? rb - 8 : rb;  // aim at 256 slices
    const uint32_t lo = std::max<uint32_t>(std::min(rb, kMinSliceBits), rb > kMaxBucketsLog2 ? rb - kMaxBucketsLog2 : 0);
    sb = std::max(sb, lo);
    sb = std::min({sb, kMaxSliceBits, rb});
    p->sb = sb;
    p->nb = 1u << (rb - sb);
    uint32_t tl = force ? 0u : g_tune_tile.load();
    if (tl == 0) tl = tuned.tile_log2;
    // 2^14-key tiles for large inputs; 2^15 when there are 2048 slices or more,
    // where a tile's segment per slice would otherwise hold only a few keys
    if (tl == 0) tl = n >= (1ull << 22) ? (p->nb >= 2048 ? 15 : 14) : 12;
    tl = std::min<uint32_t>(std::max<uint32_t>(tl, 12), 15);
    p->tile_log2 = tl;
    p->tile_keys = 1u << tl;
    p->nt = static_cast<uint32_t>((n + p->tile_keys - 1) >> tl);
    p->off_binfo = kHeaderBytes;
    p->off_table = align256(p->off_binfo + 24ull * p->nb);
    p->off_staging = align256(p->off_table + 4ull * p->nt * (p->nb + 1));
    p->bytes = align256(p->off_staging + 4ull * p->nt * p->tile_keys + kStagingPad);
    // Emit through an HBM bit-vector when it is small next to the keys
    // (R/8 <= 2n): the bit-vector round trip costs 2R/8 bytes, and in return
    // the emission runs at full occupancy instead of beside a 2^sb-bit slice.
    uint32_t path = force ? 0u : g_tune_path.load();
    if (path == 0) path = tuned.emit_path;
    const uint64_t bv_bytes = (1ull << rb) / 8u;
    if ((1u << (sb - 5)) >= kChunkWords && (path == 2 || path == 4 || (path == 0 && bv_bytes <= 2 * n))) {
      p->via_bitvec = true;
      p->n_chunks = (1ull << (rb - 5)) / kChunkWords;
      p->off_bitvec = p->bytes;
      p->off_chunk = align256(p->off_bitvec + bv_bytes);
      p->bytes = align256(p->off_chunk + 8ull * p->n_chunks);
      // Path 4 (asked for: it pays on skewed keys, where a few slices hold
      // several times the mean, and costs a table read on even ones):
      // heavy slices are shared out.  Enough tiles to cut a heavy slice into
      // chunks; its control words and kSplitMax * kSplitParts partial slices.
      if (path == 4 && p->nt >= 2u * kSplitMinTiles && p->nb >= 2u) {
        p->split = true;
        p->off_split_ctl = p->bytes;
        p->off_partials = align256(p->off_split_ctl + 4ull * kSplitCtlWords);
        p->bytes = align256(p->off_partials + 4ull * kSplitMax * kSplitParts * (1ull << (sb - 5)));
      }
    }
    // About one key per word or fewer: the slice kernel also keeps a summary
    // bit per word and its emission reads only nonzero words.  Needs the full
    // 2^20-bit slice, whose 1024 summary words give every lane of the sixteen
    // waves one.  Path 1 forces the plain word scan, path 3 the summary.
    if (!p->via_bitvec && sb == kMaxSliceBits && (path == 3 || (path == 0 && 32ull * n <= (1ull << rb))))
      p->sparse = true;
    // A tile's segment for one slice holds about tile_keys * 2^sb / R keys
    // (uniform keys).  At 8 or fewer, 64-key units would leave most lanes of
    // every load idle and take four times the batches: gather 16-key units.
    p->short_units = (static_cast<uint64_t>(p->tile_keys) << sb) <= (8ull << rb);
  }
  p->stage_cap = stage_cap_for(p->sb);
  p->slice_lds = slice_lds_bytes(p->sb, p->stage_cap);
}

int check_args(const uint32_t* keys, uint64_t n, uint32_t rb, const uint32_t* out) {
  if (rb > 32) return BITSORT_ERR_INVALID_ARG;
  if (n > 0 && (keys == nullptr || out == nullptr)) return BITSORT_ERR_INVALID_ARG;
  if (n >= (1ull << 32)) return BITSORT_ERR_TOO_LARGE;
  if (n > (1ull << rb)) return BITSORT_ERR_TOO_LARGE;
  if (n > 0 && keys != out) {
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(keys), a1 = a0 + 4 * n;
    const uintptr_t b0 = reinterpret_cast<uintptr_t>(out), b1 = b0 + 4 * n;
    if (a0 < b1 && b0 < a1) return BITSORT_ERR_INVALID_ARG;
  }
  return BITSORT_OK;
}

std::once_flag g_attr_once;
hipError_t g_attr_err = hipSuccess;

template <typename K>
void set_lds_attr(K kernel, uint32_t bytes) {
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           static_cast<int>(bytes));
  if (e != hipSuccess && g_attr_err == hipSuccess) g_attr_err = e;
}

int init_kernels() {
  std::call_once(g_attr_once, [] {
    set_lds_attr(k_partition<1024, 4>, kLdsBytes);
    set_lds_attr(k_partition<512, 16>, kLdsBytes);
    set_lds_attr(k_partition<1024, 16>, kLdsBytes);
    set_lds_attr(k_partition<1024, 32>, kLdsBytes);
    set_lds_attr(k_slice<kSliceBlock, kSliceUnroll, false, 64>, kLdsBytes);
    set_lds_attr(k_slice<kSliceBlock, kSliceUnroll, true, 64>, kLdsBytes);
    set_lds_attr(k_slice<kSliceBlock, kSliceUnroll, false, 16>, kLdsBytes);
    set_lds_attr(k_slice<kSliceBlock, kSliceUnroll, true, 16>, kLdsBytes);
    set_lds_attr(k_slice_split<kSliceBlock, kSliceUnroll, 16>, kLdsBytes);
    set_lds_attr(k_slice_split<kSliceBlock, kSliceUnroll, 64>, kLdsBytes);
    set_lds_attr(k_slice_seq<kSliceBlock, kSliceUnroll, 16>, kLdsBytes);
    set_lds_attr(k_slice_seq<kSliceBlock, kSliceUnroll, 64>, kLdsBytes);
    set_lds_attr(k_direct<kDirectBlock>, kLdsBytes);
    set_lds_attr(k_count_slice<kSliceBlock, kSliceUnroll>, kLdsBytes);
    set_lds_attr(k_partition_multi<256>, kLdsBytes);
    set_lds_attr(k_partition_multi<1024>, kLdsBytes);
    set_lds_attr(k_slice_multi<kSliceBlock, kSliceUnroll>, kLdsBytes);
    set_lds_attr(k_batch_run<256>, kLdsBytes);
    set_lds_attr(k_batch_run<512>, kLdsBytes);
    set_lds_attr(k_batch_run<1024>, kLdsBytes);
    set_lds_attr(k_partition_kv<1024, 4>, kLdsBytes);
    set_lds_attr(k_partition_kv<1024, 16>, kLdsBytes);
    set_lds_attr(k_partition_kv<1024, 32>, kLdsBytes);
    set_lds_attr(k_slice_kv<kSliceBlock, kSliceUnroll, 16>, kLdsBytes);
    set_lds_attr(k_slice_kv<kSliceBlock, kSliceUnroll, 64>, kLdsBytes);
  });
  return g_attr_err == hipSuccess ? BITSORT_OK : BITSORT_ERR_HIP;
}

int launch_status() {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? BITSORT_OK : BITSORT_ERR_HIP;
}

// Kernel timing (bitsort_profile_*): events bracketing each launch.
enum KernelId : int {
  kKPartition = 0, kKSlice, kKEmit, kKFinish, kKDirect, kKBatchPlan, kKBatchRun, kKRadixHist, kKRadixScan,
  kKRadixPass, kKCountSlice, kKPartitionMulti, kKSliceMulti, kKEmitMulti, kKFinishMulti, kKMarkAtomic,
  kKChunkCount, kKChunkScan, kKPairsScatter, kKPairsGather, kKPartitionKV, kKSliceKV, kKPairsFinish, kKCount
};
const char* const kKernelNames[kKCount] = {"k_partition", "k_slice",      "k_emit",       "k_finish",
                                           "k_direct",    "k_batch_plan", "k_batch_run",  "k_radix_hist",
                                           "k_radix_scan", "k_radix_pass", "k_count_slice",
                                           "k_partition_multi", "k_slice_multi", "k_emit_multi",
                                           "k_finish_multi", "k_mark_atomic", "k_chunk_count", "k_chunk_scan",
                                           "k_pairs_scatter", "k_pairs_gather", "k_partition_kv", "k_slice_kv",
                                           "k_pairs_finish"};
struct PendingTiming {
  int kernel;
  hipEvent_t start, stop;
};
std::atomic<bool> g_prof_on{false};
thread_local bool t_capturing = false;  // enqueueing into a graph capture or the no-allocation call: no timing events
std::mutex g_prof_mu;
std::vector<PendingTiming> g_prof_pending;
uint64_t g_prof_launches[kKCount] = {};
double g_prof_ms[kKCount] = {};

// Records the start event of a timed launch (no-op while profiling is off).
struct LaunchTimer {
  int kernel;
  hipStream_t stream;
  hipEvent_t start = nullptr;
  LaunchTimer(int k, hipStream_t s) : kernel(k), stream(s) {
    if (!g_prof_on.load(std::memory_order_relaxed) || t_capturing) return;
    if (hipEventCreate(&start) != hipSuccess || hipEventRecord(start, stream) != hipSuccess) start = nullptr;
  }
  ~LaunchTimer() {
    if (start == nullptr) return;
    hipEvent_t stop = nullptr;
    if (hipEventCreate(&stop) != hipSuccess || hipEventRecord(stop, stream) != hipSuccess) {
      (void)hipEventDestroy(start);
      if (stop) (void)hipEventDestroy(stop);
      return;
    }
    std::lock_guard<std::mutex> lock(g_prof_mu);
    g_prof_pending.push_back({kernel, start, stop});
  }
};

// Enqueue the plain path.  mode != kEmit writes the debug dumps instead.
// Partition launch shared by the bitmap and the counting path.
int launch_partition(const Plan& p, const uint32_t* keys, uint64_t n, uint32_t* staging, uint32_t* table,
                     hipStream_t stream, uint32_t* split_ctl = nullptr, Status* status = nullptr) {
  const uint64_t range = 1ull << p.rb;
  const int vec_ok = (reinterpret_cast<uintptr_t>(keys) % 16u) == 0 ? 1 : 0;
  const size_t part_lds = 4ull * (32 + round_up4(p.nb) + p.tile_keys);
  LaunchTimer timer(kKPartition, stream);
  switch (p.tile_log2) {
    case 12:  // 4096-key tiles: 1024 threads of 4 keys, so that a small input's few tiles still fill the CUs
      hipLaunchKernelGGL((k_partition<1024, 4>), dim3(p.nt), dim3(1024), part_lds, stream, keys, n, range, p.sb,
                         p.nb, staging, table, vec_ok, p.bias, split_ctl, status);
      break;
    case 13:
      hipLaunchKernelGGL((k_partition<512, 16>), dim3(p.nt), dim3(512), part_lds, stream, keys, n, range, p.sb, p.nb,
                         staging, table, vec_ok, p.bias, split_ctl, status);
      break;
    case 14:
      hipLaunchKernelGGL((k_partition<1024, 16>), dim3(p.nt), dim3(1024), part_lds, stream, keys, n, range, p.sb,
                         p.nb, staging, table, vec_ok, p.bias, split_ctl, status);
      break;
    default:
      hipLaunchKernelGGL((k_partition<1024, 32>), dim3(p.nt), dim3(1024), part_lds, stream, keys, n, range, p.sb,
                         p.nb, staging, table, vec_ok, p.bias, split_ctl, status);
      break;
  }
  return launch_status();
}

// Compute units of the current device (cached per device).
uint32_t device_cus() {
  static std::atomic<int> cached[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256u;
  int c = cached[dev].load(std::memory_order_relaxed);
  if (c <= 0) {
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
    cached[dev].store(c, std::memory_order_relaxed);
  }
  return static_cast<uint32_t>(c);
}

// status_to: where the call's status goes (the workspace header when null).
// defer_finish: the caller reads the status through the library
// (read_plain_status), so the two-kernel path leaves its finish step pending
// in the workspace header instead of launching it.
int run_plain(const Plan& p, const uint32_t* keys, uint64_t n, uint32_t* out, void* ws,
              hipStream_t stream, int mode, uint32_t* dbg_bitmap, uint64_t* dbg_prefix,
              Status* status_to = nullptr, bool defer_finish = false) {
  int rc = init_kernels();
  if (rc != BITSORT_OK) return rc;
  char* base = static_cast<char*>(ws);
  Status* status = status_to != nullptr ? status_to : reinterpret_cast<Status*>(base);
  const uint64_t range = 1ull << p.rb;
  if (p.direct) {
    LaunchTimer timer(kKDirect, stream);
    hipLaunchKernelGGL(k_direct<kDirectBlock>, dim3(1), dim3(kDirectBlock), p.slice_lds, stream, keys, n,
                       range, p.sb, p.stage_cap, out, status, mode, dbg_bitmap, dbg_prefix, p.bias);
    return launch_status();
  }
  uint32_t* table = reinterpret_cast<uint32_t*>(base + p.off_table);
  uint32_t* staging = reinterpret_cast<uint32_t*>(base + p.off_staging);
  uint64_t* info = reinterpret_cast<uint64_t*>(base + p.off_binfo);
  const bool split = p.split && mode == kEmit;
  uint32_t* split_ctl = split ? reinterpret_cast<uint32_t*>(base + p.off_split_ctl) : nullptr;
  rc = launch_partition(p, keys, n, staging, table, stream, split_ctl, status);
  if (rc != BITSORT_OK) return rc;
  uint32_t* bitvec = reinterpret_cast<uint32_t*>(base + p.off_bitvec);
  uint64_t* chunk_base = reinterpret_cast<uint64_t*>(base + p.off_chunk);
  if (p.via_bitvec && mode == kDumpBitmap) bitvec = dbg_bitmap;  // the mark step's bit-vector is the dump
  const bool defer = defer_finish && mode == kEmit && status_to == nullptr;
  Status* pending = defer ? status : nullptr;
  {
    LaunchTimer timer(kKSlice, stream);
    const uint32_t cus = device_cus();
    if (split) {
      // bit-vector route: slices of more than four times the mean (and 2^16
      // keys or more) are shared out among the workgroups that finish early
      const uint32_t grid = 8u * ((p.nb + 7u) / 8u);
      const uint64_t heavy = std::max<uint64_t>(4 * ((n + p.nb - 1) / p.nb), 1ull << 16);
      auto kernel = p.short_units ? k_slice_split<kSliceBlock, kSliceUnroll, 16>
                                  : k_slice_split<kSliceBlock, kSliceUnroll, 64>;
      hipLaunchKernelGGL(kernel, dim3(grid), dim3(kSliceBlock), p.slice_lds, stream, staging, table, p.nt,
                         p.tile_keys, p.sb, p.nb, info, bitvec, chunk_base, split_ctl,
                         reinterpret_cast<uint32_t*>(base + p.off_partials), heavy, n, out, pending, status);
      rc = launch_status();
    } else if (p.sparse && mode == kEmit && p.nb > cus) {
      // many sparse slices: one workgroup per CU (a multiple of 8), each
      // taking every (grid/8)-th slice of its XCD's run
      const uint32_t grid = std::max(8u, cus & ~7u);
      auto kernel = p.short_units ? k_slice_seq<kSliceBlock, kSliceUnroll, 16> : k_slice_seq<kSliceBlock, kSliceUnroll, 64>;
      hipLaunchKernelGGL(kernel, dim3(grid), dim3(kSliceBlock), p.slice_lds, stream, staging, table, p.nt,
                         p.tile_keys, p.sb, p.nb, out, info, 0u - p.bias, n, p.stage_cap, pending);
      rc = launch_status();
    } else {
    const uint32_t grid = 8u * ((p.nb + 7u) / 8u);
    auto kernel = p.sparse ? (p.short_units ? k_slice<kSliceBlock, kSliceUnroll, true, 16>
                                            : k_slice<kSliceBlock, kSliceUnroll, true, 64>)
                           : (p.short_units ? k_slice<kSliceBlock, kSliceUnroll, false, 16>
                                            : k_slice<kSliceBlock, kSliceUnroll, false, 64>);
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(kSliceBlock), p.slice_lds, stream, staging, table, p.nt,
                       p.tile_keys, p.sb, p.nb, p.stage_cap, out, info,
                       p.via_bitvec ? static_cast<int>(kToBitVector) : mode, dbg_bitmap, dbg_prefix, bitvec,
                       chunk_base, 0u - p.bias, n, pending);
    rc = launch_status();
    }
  }
  if (rc != BITSORT_OK || mode == kDumpBitmap || (mode == kDumpPrefix && !p.via_bitvec)) return rc;
  if (p.via_bitvec) {
    LaunchTimer timer(kKEmit, stream);
    hipLaunchKernelGGL((k_emit<kEmitBlock>), dim3(static_cast<uint32_t>(p.n_chunks)), dim3(kEmitBlock), 0, stream,
                       bitvec, chunk_base, out, mode, dbg_prefix, 0u - p.bias, nullptr);
    rc = launch_status();
    if (rc != BITSORT_OK || mode != kEmit) return rc;
  }
  if (defer) return BITSORT_OK;
  LaunchTimer timer(kKFinish, stream);
  hipLaunchKernelGGL((k_finish<kSliceBlock>), dim3(1), dim3(kSliceBlock), 0, stream, n, p.nb, info, status, out,
                     split ? BITSORT_STATUS_TIMEOUT : 0u);
  return launch_status();
}

// ---- multiset (counting) sort --------------------------------------------------

// Slices of 2^sb counters (10 <= sb <= 15) and at most 2^12 of them, so
// range_bits <= 27; tiles as for the bitmap.
void make_count_plan(uint64_t n, uint32_t rb, Plan* p) {
  *p = Plan();
  p->rb = rb;
  p->direct = false;
  uint32_t sb = rb > 8 ? rb - 8 : rb;
  sb = std::max({sb, kCountMinSliceBits, rb > kMaxBucketsLog2 ? rb - kMaxBucketsLog2 : 0u});
  sb = std::min(sb, kCountMaxSliceBits);
  p->sb = sb;
  p->nb = rb > sb ? 1u << (rb - sb) : 1u;
  p->tile_log2 = n >= (1ull << 22) ? 14 : 12;
  p->tile_keys = 1u << p->tile_log2;
  p->nt = static_cast<uint32_t>((n + p->tile_keys - 1) >> p->tile_log2);
  p->off_binfo = kHeaderBytes;
  p->off_table = align256(p->off_binfo + 24ull * p->nb);
  p->off_staging = align256(p->off_table + 4ull * p->nt * (p->nb + 1));
  p->bytes = align256(p->off_staging + 4ull * p->nt * p->tile_keys);
  p->slice_lds = 4ull * (64 + (kSliceBlock / kWave) * kWave + (1u << sb) +
                         (kSliceBlock / kWave) * (kCountWindow + 4u));
}

int run_count(const Plan& p, const uint32_t* keys, uint64_t n, uint32_t* out, void* ws, hipStream_t stream) {
  int rc = init_kernels();
  if (rc != BITSORT_OK) return rc;
  char* base = static_cast<char*>(ws);
  Status* status = reinterpret_cast<Status*>(base);
  uint32_t* table = reinterpret_cast<uint32_t*>(base + p.off_table);
  uint32_t* staging = reinterpret_cast<uint32_t*>(base + p.off_staging);
  uint64_t* info = reinterpret_cast<uint64_t*>(base + p.off_binfo);
  if ((rc = launch_partition(p, keys, n, staging, table, stream)) != BITSORT_OK) return rc;
  {
    LaunchTimer timer(kKCountSlice, stream);
    const uint32_t grid = 8u * ((p.nb + 7u) / 8u);
    hipLaunchKernelGGL((k_count_slice<kSliceBlock, kSliceUnroll>), dim3(grid), dim3(kSliceBlock), p.slice_lds,
                       stream, staging, table, p.nt, p.tile_keys, p.sb, p.nb, out, info);
    if ((rc = launch_status()) != BITSORT_OK) return rc;
  }
  LaunchTimer timer(kKFinish, stream);
  hipLaunchKernelGGL((k_finish<kSliceBlock>), dim3(1), dim3(kSliceBlock), 0, stream, n, p.nb, info, status, out,
                     0u);
  return launch_status();
}

// ---- many arrays through the plain path in one launch per kernel -------------

// Workspace of a multi launch: [header][status x count][descriptors]
// [slice info][tile tables][staging][bit-vectors][chunk prefixes].
struct MultiPlan {
  std::vector<MultiDesc> desc;
  uint32_t tiles = 0, slices = 0, chunks = 0, max_nb = 1, max_sb = kMinSliceBits, tile_log2 = 12;
  uint64_t table_words = 0, bitvec_words = 0;
  size_t off_status = 0, off_desc = 0, off_info = 0, off_table = 0, off_staging = 0, off_bitvec = 0, off_chunk = 0,
         bytes = 0;
};

int check_multi_args(const uint32_t* const* keys, const uint64_t* n, const uint8_t* range_bits,
                     uint32_t* const* out, uint32_t count) {
  if (count == 0 || count > BITSORT_BATCH_MAX_SEGMENTS || keys == nullptr || n == nullptr ||
      range_bits == nullptr || out == nullptr)
    return BITSORT_ERR_INVALID_ARG;
  for (uint32_t a = 0; a < count; ++a) {
    int rc = check_args(keys[a], n[a], range_bits[a], out[a]);
    if (rc != BITSORT_OK) return rc;
  }
  return BITSORT_OK;
}

// Per array: 2^split slices of 2^sb bits (sb in [10, 20], at most 4096
// slices), tiles of 2^tile_log2 keys.  split is set per launch, the smallest
// of 0..8 that gives the launch 256 slices or more (one per CU): few wide
// slices mean few table rows to walk and little fixed cost per key, as on the
// single-array path with its 2^20-bit slices.  Tiles hold 2^14 keys when the
// arrays have 64 slices or more on average (weighted by keys), so that a
// tile's run of keys per slice stays long, and 2^12 otherwise, where the
// smaller workgroups partition faster.  A range of 2^21 or more whose
// bit-vector is at most twice the keys' bytes (R/8 <= 2n) emits through the
// HBM bit-vector, as on the single-array path; such an array takes a split of
// 4 or more (measured best) and slices of at least one emission chunk (2^15
// bits).
// Launch limits of the multi kernels: a grid holds at most 2^32 work-items
// (HSA dispatch sizes are 32-bit), so tiles and slices stay below 2^22
// workgroups of up to 1024 threads and chunks below 2^24 of 256; the
// descriptors' first-tile, first-slice and first-chunk fields are 32-bit.
constexpr uint64_t kMultiMaxTiles = (1ull << 22) - 8;
constexpr uint64_t kMultiMaxSlices = (1ull << 22) - 8;
constexpr uint64_t kMultiMaxChunks = (1ull << 24) - 1;

// Returns BITSORT_ERR_TOO_LARGE, before any field of *p is used, when the
// arrays together pass a launch limit; the sums are taken in 64 bits.
int make_multi_plan(const uint32_t* const* keys, const uint64_t* n, const uint8_t* range_bits,
                    uint32_t* const* out, uint32_t count, MultiPlan* p) {
  *p = MultiPlan();
  auto via_bitvec = [&](uint32_t a) {
    const uint32_t rb = range_bits[a];
    return rb >= 21 && (1ull << rb) / 8u <= 2 * n[a];
  };
  auto slice_bits = [&](uint32_t a, uint32_t split) {
    const uint32_t rb = range_bits[a];
    uint32_t sb = rb > split ? rb - split : 0u;
    if (via_bitvec(a)) sb = std::max(rb - std::max(split, 4u), kChunkLog2Bits);
    sb = std::max({sb, kMinSliceBits, rb > kMaxBucketsLog2 ? rb - kMaxBucketsLog2 : 0u});
    return std::min(sb, kMaxSliceBits);
  };
  uint32_t split = 0;
  for (; split < 8; ++split) {
    uint64_t slices = 0;
    for (uint32_t a = 0; a < count; ++a) {
      const uint32_t sb = slice_bits(a, split);
      slices += range_bits[a] > sb ? 1ull << (range_bits[a] - sb) : 1u;
    }
    if (slices >= 256) break;
  }
  uint64_t total = 0, weighted = 0;
  for (uint32_t a = 0; a < count; ++a) {
    const uint32_t sb = slice_bits(a, split);
    total += n[a];
    weighted += n[a] << (range_bits[a] > sb ? range_bits[a] - sb : 0u);
  }
  p->tile_log2 = weighted >= 64 * total && total > 0 ? 14u : 12u;
  const uint64_t tile_keys = 1ull << p->tile_log2;
  {
    uint64_t tiles = 0, slices = 0, chunks = 0;
    for (uint32_t a = 0; a < count; ++a) {
      const uint32_t rb = range_bits[a], sb = slice_bits(a, split);
      tiles += (n[a] + tile_keys - 1) / tile_keys;
      slices += rb > sb ? 1ull << (rb - sb) : 1ull;
      if (via_bitvec(a)) chunks += 1ull << (rb - kChunkLog2Bits);
    }
    if (tiles > kMultiMaxTiles || slices > kMultiMaxSlices || chunks > kMultiMaxChunks) return BITSORT_ERR_TOO_LARGE;
  }
  p->desc.resize(count);
  for (uint32_t a = 0; a < count; ++a) {
    MultiDesc& d = p->desc[a];
    const uint32_t rb = range_bits[a];
    const uint32_t sb = slice_bits(a, split);
    d.via_bitvec = via_bitvec(a) ? 1u : 0u;
    d.keys = keys[a];
    d.out = out[a];
    d.n = n[a];
    d.rb = rb;
    d.sb = sb;
    d.nb = rb > sb ? 1u << (rb - sb) : 1u;
    d.nt = static_cast<uint32_t>((n[a] + tile_keys - 1) / tile_keys);
    d.tile0 = p->tiles;
    d.slice0 = p->slices;
    d.table_off = p->table_words;
    p->tiles += d.nt;
    p->slices += d.nb;
    p->table_words += static_cast<uint64_t>(d.nt) * (d.nb + 1);
    d.chunk0 = p->chunks;
    d.bitvec_off = p->bitvec_words;
    if (d.via_bitvec) {
      p->chunks += 1u << (rb - kChunkLog2Bits);
      p->bitvec_words += 1ull << (rb - 5);
    }
    p->max_nb = std::max(p->max_nb, d.nb);
    p->max_sb = std::max(p->max_sb, d.sb);
  }
  size_t o = kHeaderBytes;
  p->off_status = o;
  o = align256(o + sizeof(SegStatus) * count);
  p->off_desc = o;
  o = align256(o + sizeof(MultiDesc) * count);
  p->off_info = o;
  o = align256(o + 24ull * p->slices);
  p->off_table = o;
  o = align256(o + 4ull * p->table_words);
  p->off_staging = o;
  o = align256(o + 4ull * p->tiles * tile_keys + kStagingPad);
  p->off_bitvec = o;
  o = align256(o + 4ull * p->bitvec_words);
  p->off_chunk = o;
  o = align256(o + 8ull * p->chunks);
  p->bytes = o;
  return BITSORT_OK;
}

// Enqueue the three multi kernels; the descriptors must already be on the
// device at ws + off_desc.
int run_multi(const MultiPlan& p, uint32_t count, void* ws, hipStream_t stream) {
  int rc = init_kernels();
  if (rc != BITSORT_OK) return rc;
  char* base = static_cast<char*>(ws);
  const MultiDesc* desc = reinterpret_cast<const MultiDesc*>(base + p.off_desc);
  uint64_t* info = reinterpret_cast<uint64_t*>(base + p.off_info);
  uint32_t* table = reinterpret_cast<uint32_t*>(base + p.off_table);
  uint32_t* staging = reinterpret_cast<uint32_t*>(base + p.off_staging);
  if (p.tiles > 0) {
    LaunchTimer timer(kKPartitionMulti, stream);
    const size_t part_lds = 4ull * (32 + round_up4(p.max_nb) + (1u << p.tile_log2));
    if (p.tile_log2 == 14)
      hipLaunchKernelGGL(k_partition_multi<1024>, dim3(p.tiles), dim3(1024), part_lds, stream, desc, count, staging,
                         table);
    else
      hipLaunchKernelGGL(k_partition_multi<256>, dim3(p.tiles), dim3(256), part_lds, stream, desc, count, staging,
                         table);
    if ((rc = launch_status()) != BITSORT_OK) return rc;
  }
  {
    LaunchTimer timer(kKSliceMulti, stream);
    const uint32_t stage_cap = stage_cap_for(p.max_sb);
    const uint32_t grid = 8u * ((p.slices + 7u) / 8u);
    hipLaunchKernelGGL((k_slice_multi<kSliceBlock, kSliceUnroll>), dim3(grid), dim3(kSliceBlock),
                       slice_lds_bytes(p.max_sb, stage_cap), stream, desc, count, p.slices, 1u << p.tile_log2,
                       staging, table, info,
                       stage_cap, reinterpret_cast<uint32_t*>(base + p.off_bitvec),
                       reinterpret_cast<uint64_t*>(base + p.off_chunk));
    if ((rc = launch_status()) != BITSORT_OK) return rc;
  }
  if (p.chunks > 0) {
    LaunchTimer timer(kKEmitMulti, stream);
    hipLaunchKernelGGL(k_emit_multi<kEmitBlock>, dim3(p.chunks), dim3(kEmitBlock), 0, stream, desc, count,
                       reinterpret_cast<const uint32_t*>(base + p.off_bitvec),
                       reinterpret_cast<const uint64_t*>(base + p.off_chunk));
    if ((rc = launch_status()) != BITSORT_OK) return rc;
  }
  LaunchTimer timer(kKFinishMulti, stream);
  hipLaunchKernelGGL(k_finish_multi<kSliceBlock>, dim3(count), dim3(kSliceBlock), 0, stream, desc, info,
                     reinterpret_cast<Status*>(base + p.off_status));
  return launch_status();
}

// Batch tuning: workgroup size of k_batch_run and bits per LDS slice.
struct BatchTuning {
  uint32_t block = 1024;
  uint32_t slice_bits = kBatchSliceBits;
};
BatchTuning g_batch_tuned;           // set by bitsort_autotune_batch_u32 / the tuning cache
std::atomic<uint32_t> g_batch_block{0};
std::atomic<uint32_t> g_batch_sb{0};

BatchTuning batch_tuning() {
  BatchTuning t;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    t = g_batch_tuned;
  }
  if (g_batch_block.load()) t.block = g_batch_block.load();
  if (g_batch_sb.load()) t.slice_bits = g_batch_sb.load();
  return t;
}

int check_batch_args(const uint32_t* keys, const uint64_t* offsets, uint32_t num_segments,
                     const uint8_t* range_bits, const uint32_t* out, uint64_t max_keys) {
  if (num_segments == 0 || num_segments > BITSORT_BATCH_MAX_SEGMENTS) return BITSORT_ERR_INVALID_ARG;
  if (keys == nullptr || offsets == nullptr || range_bits == nullptr || out == nullptr) return BITSORT_ERR_INVALID_ARG;
  if (max_keys >= (1ull << 40)) return BITSORT_ERR_TOO_LARGE;
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(keys), a1 = a0 + 4 * max_keys;
  const uintptr_t b0 = reinterpret_cast<uintptr_t>(out), b1 = b0 + 4 * max_keys;
  if (max_keys > 0 && a0 < b1 && b0 < a1) return BITSORT_ERR_INVALID_ARG;
  return BITSORT_OK;
}

size_t batch_workspace_bytes(uint32_t num_segments, const BatchTuning& t) {
  const uint64_t max_items = static_cast<uint64_t>(num_segments) << (kMaxBatchRangeBits - t.slice_bits);
  const size_t off_items = align256(kHeaderBytes + sizeof(SegStatus) * num_segments);
  return align256(off_items + sizeof(uint2) * max_items);
}

template <int BLOCK>
int launch_batch_run(const uint32_t* keys, const uint64_t* offsets, const uint8_t* range_bits, uint32_t sbb,
                     const uint2* items, uint32_t* counter, uint32_t* out, SegStatus* st, uint64_t max_items,
                     hipStream_t s) {
  const uint32_t stage_cap = stage_cap_for(sbb);
  const size_t lds = slice_lds_bytes(sbb, stage_cap);
  int cus = 256, dev = 0, per_cu = 1;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_run<BLOCK>, BLOCK, lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const uint64_t grid = std::min<uint64_t>(static_cast<uint64_t>(cus) * per_cu, max_items);
  LaunchTimer timer(kKBatchRun, s);
  hipLaunchKernelGGL(k_batch_run<BLOCK>, dim3(static_cast<uint32_t>(grid)), dim3(BLOCK), lds, s, keys, offsets,
                     range_bits, sbb, stage_cap, items, counter, out, st);
  return launch_status();
}

// Enqueue the batch: plan on the device, then the persistent item loop.
int run_batch(const uint32_t* keys, const uint64_t* offsets, uint32_t num_segments, const uint8_t* range_bits,
              uint32_t* out, uint64_t max_keys, void* ws, hipStream_t s, const BatchTuning& t) {
  const uint32_t sbb = t.slice_bits;
  const uint64_t max_items = static_cast<uint64_t>(num_segments) << (kMaxBatchRangeBits - sbb);
  const size_t off_items = align256(kHeaderBytes + sizeof(SegStatus) * num_segments);
  char* base = static_cast<char*>(ws);
  uint32_t* counter = reinterpret_cast<uint32_t*>(base);
  SegStatus* st = reinterpret_cast<SegStatus*>(base + kHeaderBytes);
  uint2* items = reinterpret_cast<uint2*>(base + off_items);
  int rc;
  {
    LaunchTimer timer(kKBatchPlan, s);
    hipLaunchKernelGGL(k_batch_plan, dim3(1), dim3(1024), 0, s, offsets, range_bits, num_segments, max_keys, sbb,
                       items, counter, st);
    rc = launch_status();
  }
  if (rc != BITSORT_OK) return rc;
  switch (t.block) {
    case 256:
      return launch_batch_run<256>(keys, offsets, range_bits, sbb, items, counter, out, st, max_items, s);
    case 512:
      return launch_batch_run<512>(keys, offsets, range_bits, sbb, items, counter, out, st, max_items, s);
    default:
      return launch_batch_run<1024>(keys, offsets, range_bits, sbb, items, counter, out, st, max_items, s);
  }
}

// Library-owned workspaces, one per (device, stream).
// ---- radix sort (the paper's Algorithm 1 in 8-bit digits) -------------------

struct RadixPlan {
  uint32_t passes = 0, hist_blocks = 1, key_bytes = 4, items = 32;
  bool pairs = false;
  uint64_t ntiles = 0, clear_words = 0;
  size_t off_tickets = 0, off_lookback = 0, off_partials = 0, off_digit = 0, off_tmp = 0, off_vtmp = 0, bytes = 0;
};

// Items per thread of k_radix_pass: 32 for 32-bit keys alone, 16 when the
// tile's LDS holds 8-byte keys or keys and values (32 KiB either way).
// Keys per thread of a radix tile (256 threads): 32 for uint32 keys, 20 for
// uint64 keys and key-value records (measured over 16..24 and 32..48).
constexpr uint32_t radix_items(uint32_t key_bytes, bool pairs) { return key_bytes == 4 && !pairs ? 32u : 20u; }

// Workspace: status header, then (cleared by k_radix_hist) one ticket per
// pass and the look-back words [passes][tiles][256], then the partial
// histograms, the digit starts, and ping-pong buffers of n keys (and values).
void make_radix_plan(uint64_t n, uint32_t key_bits, uint32_t key_bytes, bool pairs, RadixPlan* p) {
  p->passes = (key_bits + 7u) / 8u;
  p->key_bytes = key_bytes;
  p->pairs = pairs;
  p->items = radix_items(key_bytes, pairs);
  const uint64_t tile = static_cast<uint64_t>(kRadixBlock) * p->items;
  p->ntiles = (n + tile - 1) / tile;
  p->hist_blocks = static_cast<uint32_t>(
      std::min<uint64_t>(kRadixHistBlocks, std::max<uint64_t>(1, (n + 1024ull * 64 - 1) / (1024ull * 64))));
  const uint32_t stride = key_bytes == 8 ? RadixTraits<uint64_t>::kPartStride : RadixTraits<uint32_t>::kPartStride;
  size_t o = kHeaderBytes;
  p->off_tickets = o;
  o = align256(o + 4ull * kRadixMaxPassesAll);
  p->off_lookback = o;
  o = align256(o + 4ull * p->passes * p->ntiles * kRadixDigits);
  p->clear_words = (o - p->off_tickets) / 4;
  p->off_partials = o;
  o = align256(o + 4ull * p->hist_blocks * stride);
  p->off_digit = o;
  o = align256(o + 4ull * kRadixMaxPassesAll * kRadixDigits);
  p->off_tmp = o;
  o = align256(o + key_bytes * n);
  p->off_vtmp = o;
  if (pairs) o = align256(o + 4ull * n);
  p->bytes = o;
}

bool overlaps(const void* a, const void* b, uint64_t bytes) {
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
  return a0 < b0 + bytes && b0 < a0 + bytes;
}

int check_radix_args(const void* keys, uint64_t n, uint32_t key_bits, uint32_t key_bytes, const void* out) {
  if (key_bits > 8 * key_bytes) return BITSORT_ERR_INVALID_ARG;
  if (n > 0 && (keys == nullptr || out == nullptr)) return BITSORT_ERR_INVALID_ARG;
  if (n > kRadixMaxN) return BITSORT_ERR_TOO_LARGE;
  if (n > 0 && keys != out && overlaps(keys, out, key_bytes * n)) return BITSORT_ERR_INVALID_ARG;
  return BITSORT_OK;
}

// Enqueue the radix sort: histogram + scan, then one launch per pass reading
// from the previous pass's buffer.  The buffers alternate between `out` and
// the workspace's tmp so that the last pass writes `out`; when an output
// aliases its input, pass 0 writes tmp and an odd pass count ends with a copy.
template <typename K, bool PAIRS>
int run_radix(const RadixPlan& p, const K* keys, const uint32_t* vals, uint64_t n, uint32_t key_bits, K flip, K* out,
              uint32_t* vout, void* ws, hipStream_t stream) {
  using T = RadixTraits<K>;
  constexpr int kItems = static_cast<int>(radix_items(sizeof(K), PAIRS));
  char* base = static_cast<char*>(ws);
  Status* status = reinterpret_cast<Status*>(base);
  uint32_t* tickets = reinterpret_cast<uint32_t*>(base + p.off_tickets);
  uint32_t* lookback = reinterpret_cast<uint32_t*>(base + p.off_lookback);
  uint32_t* partials = reinterpret_cast<uint32_t*>(base + p.off_partials);
  uint32_t* digit = reinterpret_cast<uint32_t*>(base + p.off_digit);
  K* tmp = reinterpret_cast<K*>(base + p.off_tmp);
  uint32_t* vtmp = reinterpret_cast<uint32_t*>(base + p.off_vtmp);
  int rc;
  {
    LaunchTimer timer(kKRadixHist, stream);
    hipLaunchKernelGGL(k_radix_hist<K>, dim3(p.hist_blocks), dim3(kRadixHistBlock), 0, stream, keys, n, key_bits,
                       p.passes, flip, partials, tickets, p.clear_words);
    if ((rc = launch_status()) != BITSORT_OK) return rc;
  }
  {
    LaunchTimer timer(kKRadixScan, stream);
    hipLaunchKernelGGL(k_radix_scan, dim3(std::max(p.passes, 1u)), dim3(kRadixHistBlock), 0, stream, partials,
                       p.hist_blocks, T::kPartStride, T::kMaxPasses * kRadixDigits, p.passes, n, digit, status);
    if ((rc = launch_status()) != BITSORT_OK) return rc;
  }
  const bool alias = static_cast<const void*>(keys) == out || (PAIRS && static_cast<const void*>(vals) == vout);
  if (p.passes == 0) {
    if (static_cast<const void*>(keys) != out &&
        hipMemcpyAsync(out, keys, sizeof(K) * n, hipMemcpyDeviceToDevice, stream) != hipSuccess)
      return BITSORT_ERR_HIP;
    if (PAIRS && vals != vout && hipMemcpyAsync(vout, vals, 4 * n, hipMemcpyDeviceToDevice, stream) != hipSuccess)
      return BITSORT_ERR_HIP;
    return BITSORT_OK;
  }
  K* bufs[2];
  uint32_t* vbufs[2];
  if (alias || p.passes % 2 == 0) {
    bufs[0] = tmp;
    bufs[1] = out;
    vbufs[0] = vtmp;
    vbufs[1] = vout;
  } else {
    bufs[0] = out;
    bufs[1] = tmp;
    vbufs[0] = vout;
    vbufs[1] = vtmp;
  }
  const K* src = keys;
  const uint32_t* vsrc = vals;
  for (uint32_t pass = 0; pass < p.passes; ++pass) {
    K* dst = bufs[pass % 2];
    uint32_t* vdst = vbufs[pass % 2];
    LaunchTimer timer(kKRadixPass, stream);
    hipLaunchKernelGGL((k_radix_pass<K, PAIRS, kItems>), dim3(static_cast<uint32_t>(p.ntiles)), dim3(kRadixBlock), 0,
                       stream, src, dst, vsrc, vdst, n, 8 * pass, radix_digit_mask(key_bits, pass), flip,
                       digit + pass * kRadixDigits, lookback + static_cast<uint64_t>(pass) * p.ntiles * kRadixDigits,
                       tickets + pass, status);
    if ((rc = launch_status()) != BITSORT_OK) return rc;
    src = dst;
    vsrc = vdst;
  }
  if (src != out && hipMemcpyAsync(out, src, sizeof(K) * n, hipMemcpyDeviceToDevice, stream) != hipSuccess)
    return BITSORT_ERR_HIP;
  if (PAIRS && vsrc != vout && hipMemcpyAsync(vout, vsrc, 4 * n, hipMemcpyDeviceToDevice, stream) != hipSuccess)
    return BITSORT_ERR_HIP;
  return BITSORT_OK;
}

struct StreamCtx {
  void* ws = nullptr;
  size_t bytes = 0;
  bool external = false;   // ws is the caller's (bitsort_set_workspace): never grown or freed here
  bool last_empty = true;  // last call had n == 0 (status is all zero)
  bool used = false;
  void* batch_ws = nullptr;
  size_t batch_bytes = 0;
  uint32_t batch_segments = 0;
  void* desc_host = nullptr;        // pinned staging of bitsort_batch_ptr_u32's descriptors
  size_t desc_host_bytes = 0;
  hipEvent_t desc_copied = nullptr;  // the last descriptor upload has left desc_host
  void* atomic_ws = nullptr;         // bitsort_u32_atomic's workspace: zero when allocated, kept zero
  size_t atomic_bytes = 0;
  bool last_atomic = false;          // the last call's status is in atomic_ws
};
std::mutex g_mu;
std::map<std::pair<int, void*>, StreamCtx> g_ctx;

StreamCtx& ctx_for(bitsort_stream_t stream) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  return g_ctx[{dev, stream}];
}

int grow(void** ptr, size_t* have, size_t need, hipStream_t stream, bool external = false) {
  if (*have >= need && *ptr != nullptr) return BITSORT_OK;
  if (external) return BITSORT_ERR_NO_MEMORY;  // the caller's workspace is too small: no allocation
  if (*ptr != nullptr) {
    if (hipStreamSynchronize(stream) != hipSuccess) return BITSORT_ERR_HIP;
    if (hipFree(*ptr) != hipSuccess) return BITSORT_ERR_HIP;
    *ptr = nullptr;
    *have = 0;
  }
  const size_t sz = std::max<size_t>(align256(need), 1 << 20);
  if (hipMalloc(ptr, sz) != hipSuccess) {
    *ptr = nullptr;
    (void)hipGetLastError();
    return BITSORT_ERR_NO_MEMORY;
  }
  *have = sz;
  return BITSORT_OK;
}

// Status of the last sort on a workspace (synchronises `stream`).  A plain
// sort that left its finish step pending gets it now: k_finish runs on the
// stream (totals, flags, compaction after a repeated key) and clears the
// pending mark, so a second read finds the final status.
int read_plain_status(void* ws, hipStream_t stream, bitsort_status_t* st) {
  if (hipStreamSynchronize(stream) != hipSuccess) return BITSORT_ERR_HIP;
  Status s{};
  if (hipMemcpy(&s, ws, sizeof(s), hipMemcpyDeviceToHost) != hipSuccess) return BITSORT_ERR_HIP;
  if (s.done == kFinishPending) {
    PendingFinish d{};
    if (hipMemcpy(&d, static_cast<char*>(ws) + kPendingOffset, sizeof(d), hipMemcpyDeviceToHost) != hipSuccess)
      return BITSORT_ERR_HIP;
    if (d.nb == 0 || d.info == nullptr) return BITSORT_ERR_INVALID_ARG;
    hipLaunchKernelGGL((k_finish<kSliceBlock>), dim3(1), dim3(kSliceBlock), 0, stream, d.n, d.nb, d.info,
                       static_cast<Status*>(ws), d.out, d.keep);
    if (launch_status() != BITSORT_OK || hipStreamSynchronize(stream) != hipSuccess) return BITSORT_ERR_HIP;
    if (hipMemcpy(&s, ws, sizeof(s), hipMemcpyDeviceToHost) != hipSuccess) return BITSORT_ERR_HIP;
  }
  st->flags = s.flags;
  st->_pad = 0;
  st->count = s.count;
  return BITSORT_OK;
}

void splitmix_keys(uint64_t seed, uint32_t k[4]) {
  uint64_t st = seed;
  for (int i = 0; i < 4; ++i) {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    k[i] = static_cast<uint32_t>(z);
  }
}

// Radix sort on the stream's library workspace (grown as needed).
template <typename K, bool PAIRS>
int radix_on_stream(const K* keys, const uint32_t* vals, uint64_t n, uint32_t key_bits, K flip, K* out, uint32_t* vout,
                    bitsort_stream_t stream) {
  int rc = check_radix_args(keys, n, key_bits, sizeof(K), out);
  if (rc != BITSORT_OK) return rc;
  if (PAIRS && n > 0) {
    if (vals == nullptr || vout == nullptr) return BITSORT_ERR_INVALID_ARG;
    if (vals != vout && overlaps(vals, vout, 4 * n)) return BITSORT_ERR_INVALID_ARG;
    if (overlaps(out, vout, 4 * n) || overlaps(keys, vout, 4 * n) || overlaps(vals, out, 4 * n))
      return BITSORT_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lock(g_mu);
  StreamCtx& c = ctx_for(stream);
  c.used = true;
  if (n == 0) {
    c.last_empty = true;
    return BITSORT_OK;
  }
  if ((rc = init_kernels()) != BITSORT_OK) return rc;
  RadixPlan p;
  make_radix_plan(n, key_bits, sizeof(K), PAIRS, &p);
  rc = grow(&c.ws, &c.bytes, p.bytes, s, c.external);
  if (rc != BITSORT_OK) return rc;
  c.last_empty = false;
  c.last_atomic = false;
  return run_radix<K, PAIRS>(p, keys, vals, n, key_bits, flip, out, vout, c.ws, s);
}

// ---- the bit-vector marked in HBM with atomics (bitsort_u32_atomic) ---------------

// Workspace: [status + marked-key counter][chunk counts u32][chunk prefixes
// u64][bit-vector, at least one 1024-word chunk], every part at the same
// offset whatever the range (room for the counts and prefixes of a 2^32-bit
// range), so that calls of different widths never write their counts into
// words of another call's bit-vector.  Zeroed once when it is allocated;
// each call leaves its bit-vector zero again (the emission clears the words
// it read, k_chunk_scan the counter), so no call clears the bit-vector in a
// pass of its own.
struct AtomicPlan {
  uint64_t words = 0, chunks = 0;
  size_t off_counts = 0, off_base = 0, off_bitvec = 0, bytes = 0;
};
constexpr size_t kAtomicCounterOffset = 128;

void make_atomic_plan(uint32_t rb, AtomicPlan* p) {
  *p = AtomicPlan();
  p->words = std::max<uint64_t>((1ull << rb) / 32u, kChunkWords);
  p->chunks = p->words / kChunkWords;
  constexpr uint64_t kMaxChunks = (1ull << 32) / 32u / kChunkWords;
  p->off_counts = kHeaderBytes;
  p->off_base = align256(p->off_counts + 4 * kMaxChunks);
  p->off_bitvec = align256(p->off_base + 8 * kMaxChunks);
  p->bytes = align256(p->off_bitvec + 4 * p->words);
}

int run_atomic(const AtomicPlan& p, const uint32_t* keys, uint64_t n, uint32_t rb, uint32_t* out, void* ws,
               hipStream_t s) {
  char* base = static_cast<char*>(ws);
  auto* status = reinterpret_cast<Status*>(base);
  auto* valid = reinterpret_cast<unsigned long long*>(base + kAtomicCounterOffset);
  auto* counts = reinterpret_cast<uint32_t*>(base + p.off_counts);
  auto* chunk_base = reinterpret_cast<uint64_t*>(base + p.off_base);
  auto* bitvec = reinterpret_cast<uint32_t*>(base + p.off_bitvec);
  const uint64_t per_block = static_cast<uint64_t>(kMarkBlock) * kMarkUnroll;
  const uint64_t grid = std::min<uint64_t>((n + per_block - 1) / per_block, 8ull * device_cus());
  {
    LaunchTimer timer(kKMarkAtomic, s);
    hipLaunchKernelGGL(k_mark_atomic<kMarkBlock>, dim3(static_cast<uint32_t>(grid)), dim3(kMarkBlock), 0, s, keys, n,
                       1ull << rb, bitvec, valid);
    if (launch_status() != BITSORT_OK) return BITSORT_ERR_HIP;
  }
  {
    LaunchTimer timer(kKChunkCount, s);
    hipLaunchKernelGGL(k_chunk_count, dim3(static_cast<uint32_t>(p.chunks)), dim3(256), 0, s, bitvec, counts);
    if (launch_status() != BITSORT_OK) return BITSORT_ERR_HIP;
  }
  {
    LaunchTimer timer(kKChunkScan, s);
    hipLaunchKernelGGL(k_chunk_scan<1024>, dim3(1), dim3(1024), 0, s, counts, p.chunks, chunk_base, n, valid,
                       status);
    if (launch_status() != BITSORT_OK) return BITSORT_ERR_HIP;
  }
  LaunchTimer timer(kKEmit, s);
  hipLaunchKernelGGL((k_emit<kEmitBlock>), dim3(static_cast<uint32_t>(p.chunks)), dim3(kEmitBlock), 0, s, bitvec,
                     chunk_base, out, static_cast<int>(kEmit), nullptr, 0u, bitvec);
  return launch_status();
}

#include "serve.inc"

// ---- the no-allocation entry point --------------------------------------------
// A fixed device array per GPU serves as the plain path's workspace for
// bitsort_u32_noalloc; the loader places one copy on every GPU the library
// runs on and it lives until the process ends.  In host code its name is a
// host-side stand-in and never a device address: kernels and copies get the
// address that hipGetSymbolAddress returns on the current device, looked up
// once per device on its first call there.
constexpr size_t kNoAllocBytes = BITSORT_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char noalloc_scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

int noalloc_scratch_of_device(void** ptr) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return BITSORT_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (g_noalloc_ptr[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch)) != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return BITSORT_ERR_HIP;
    }
    g_noalloc_ptr[dev] = p;
  }
  *ptr = g_noalloc_ptr[dev];
  return BITSORT_OK;
}

// Enqueue a pointer-array launch planned in p: its workspace is the stream's
// batch workspace, its descriptors go up from the stream's pinned buffer.
// Called with g_mu held.
int multi_on_stream(StreamCtx& c, const MultiPlan& p, uint32_t count, hipStream_t s) {
  int rc = grow(&c.batch_ws, &c.batch_bytes, p.bytes, s);
  if (rc != BITSORT_OK) return rc;
  c.batch_segments = count;
  // Descriptors go up from a pinned buffer of the stream's own; before it is
  // refilled, the previous upload from it must have finished.
  const size_t dbytes = sizeof(MultiDesc) * count;
  if (c.desc_copied != nullptr && hipEventSynchronize(c.desc_copied) != hipSuccess) return BITSORT_ERR_HIP;
  if (c.desc_copied == nullptr && hipEventCreateWithFlags(&c.desc_copied, hipEventDisableTiming) != hipSuccess) {
    c.desc_copied = nullptr;
    return BITSORT_ERR_HIP;
  }
  if (c.desc_host_bytes < dbytes) {
    if (c.desc_host != nullptr) (void)hipHostFree(c.desc_host);
    c.desc_host = nullptr;
    c.desc_host_bytes = 0;
    if (hipHostMalloc(&c.desc_host, dbytes, hipHostMallocDefault) != hipSuccess) {
      c.desc_host = nullptr;
      return BITSORT_ERR_NO_MEMORY;
    }
    c.desc_host_bytes = dbytes;
  }
  std::memcpy(c.desc_host, p.desc.data(), dbytes);
  if (hipMemcpyAsync(static_cast<char*>(c.batch_ws) + p.off_desc, c.desc_host, dbytes, hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipEventRecord(c.desc_copied, s) != hipSuccess)
    return BITSORT_ERR_HIP;
  return run_multi(p, count, c.batch_ws, s);
}


// ---- uint64 keys over ranges up to 2^36 (bitsort_u64) -------------------------

// Workspace of bitsort_u64 (the stream's plain workspace): [status][tile
// table u32 nt x bins][tile starts u32 nt x bins][bin totals u64][group ->
// array index i32][low 32-bit keys, n].  The pointer-array launch over the
// groups uses the stream's batch workspace.
int run_wide(StreamCtx& c, const uint64_t* keys, uint64_t n, uint32_t rb, uint64_t* out, hipStream_t s) {
  const uint64_t nt = (n + kWideTile - 1) / kWideTile;
  const size_t off_table = kHeaderBytes;
  const size_t off_starts = align256(off_table + 4ull * nt * kWideBins);
  const size_t off_totals = align256(off_starts + 4ull * nt * kWideBins);
  const size_t off_present = align256(off_totals + 8ull * kWideBins);
  const size_t off_low = align256(off_present + 4ull * kWideGroups);
  const size_t bytes = align256(off_low + 4ull * n);
  int rc = grow(&c.ws, &c.bytes, bytes, s, c.external);
  if (rc != BITSORT_OK) return rc;
  char* base = static_cast<char*>(c.ws);
  auto* table = reinterpret_cast<uint32_t*>(base + off_table);
  auto* starts = reinterpret_cast<uint32_t*>(base + off_starts);
  auto* totals = reinterpret_cast<uint64_t*>(base + off_totals);
  auto* present = reinterpret_cast<int32_t*>(base + off_present);
  auto* low = reinterpret_cast<uint32_t*>(base + off_low);
  hipLaunchKernelGGL(k_wide_count, dim3(static_cast<uint32_t>(nt)), dim3(kWideBlock), 0, s, keys, n, rb, table);
  hipLaunchKernelGGL(k_wide_scan, dim3(kWideBins), dim3(1024), 0, s, table, nt, starts, totals);
  hipLaunchKernelGGL(k_wide_split, dim3(static_cast<uint32_t>(nt)), dim3(kWideBlock), 0, s, keys, n, rb, starts,
                     totals, low);
  if ((rc = launch_status()) != BITSORT_OK) return rc;
  // The groups' sizes plan the pointer-array launch: the host waits here.
  uint64_t tot[kWideBins] = {};
  if (hipMemcpyAsync(tot, totals, sizeof(tot), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return BITSORT_ERR_HIP;
  std::vector<const uint32_t*> gk;
  std::vector<uint32_t*> go;
  std::vector<uint64_t> gn;
  std::vector<uint8_t> grb;
  int32_t idx[kWideGroups];
  uint64_t kept = 0;
  for (uint32_t g = 0; g < kWideGroups; ++g) {
    idx[g] = -1;
    if (tot[g] > 0) {
      idx[g] = static_cast<int32_t>(gk.size());
      gk.push_back(low + kept);
      go.push_back(low + kept);  // sorted in place
      gn.push_back(tot[g]);
      grb.push_back(static_cast<uint8_t>(rb > 32 ? 32 : rb));
    }
    kept += tot[g];
  }
  if (hipMemcpy(present, idx, sizeof(idx), hipMemcpyHostToDevice) != hipSuccess) return BITSORT_ERR_HIP;
  const SegStatus* seg = nullptr;
  if (!gk.empty()) {
    MultiPlan mp;
    const uint32_t count = static_cast<uint32_t>(gk.size());
    if ((rc = make_multi_plan(gk.data(), gn.data(), grb.data(), go.data(), count, &mp)) != BITSORT_OK) return rc;
    if ((rc = multi_on_stream(c, mp, count, s)) != BITSORT_OK) return rc;
    seg = reinterpret_cast<const SegStatus*>(static_cast<char*>(c.batch_ws) + mp.off_status);
  }
  const uint64_t blocks = std::max<uint64_t>(1, std::min<uint64_t>((kept + 255) / 256, 8ull * device_cus()));
  hipLaunchKernelGGL(k_wide_join, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, low, totals, present, seg,
                     kept, out, reinterpret_cast<Status*>(base));
  return launch_status();
}
}  // namespace

// ---------------------------------------------------------------------------
// C ABI.

extern "C" {

int bitsort_version(void) { return 10000; }

const char* bitsort_error_string(int code) {
  switch (code) {
    case BITSORT_OK: return "ok";
    case BITSORT_ERR_INVALID_ARG: return "invalid argument";
    case BITSORT_ERR_TOO_LARGE: return "problem too large (n > 2^range_bits, n >= 2^32, or a stated limit)";
    case BITSORT_ERR_NO_MEMORY: return "out of device memory or workspace too small";
    case BITSORT_ERR_HIP: return "HIP runtime error";
    default: return "unknown error";
  }
}

size_t bitsort_workspace_bytes(uint64_t n, uint32_t range_bits) {
  if (range_bits > 32 || n >= (1ull << 32) || n > (1ull << range_bits)) return 0;
  Plan p;
  make_plan(n, range_bits, &p);
  return p.bytes;
}

int bitsort_u32_ws(const uint32_t* keys, uint64_t n, uint32_t range_bits, uint32_t* out, void* workspace,
                   size_t ws_bytes, bitsort_stream_t stream) {
  int rc = check_args(keys, n, range_bits, out);
  if (rc != BITSORT_OK) return rc;
  if (workspace == nullptr || (reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return BITSORT_ERR_INVALID_ARG;
  Plan p;
  make_plan(n, range_bits, &p);
  if (ws_bytes < p.bytes) return BITSORT_ERR_NO_MEMORY;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n == 0) {  // a zero status; a fill kernel, not a memset: the call may be stream-captured
    hipLaunchKernelGGL(serve::k_fill_u64, dim3(1), dim3(64), 0, s, static_cast<unsigned long long*>(workspace), 2u);
    return launch_status();
  }
  return run_plain(p, keys, n, out, workspace, s, kEmit, nullptr, nullptr, nullptr, true);
}

int bitsort_u32_noalloc(const uint32_t* keys, uint64_t n, uint32_t range_bits, uint32_t* out,
                        bitsort_status_t* status, bitsort_stream_t stream) {
  int rc = check_args(keys, n, range_bits, out);
  if (rc != BITSORT_OK) return rc;
  if (status != nullptr) {
    if ((reinterpret_cast<uintptr_t>(status) & 7u) != 0) return BITSORT_ERR_INVALID_ARG;
    auto meets = [&](const void* a) {  // [status, status + 16) against [a, a + 4n)
      const uintptr_t s0 = reinterpret_cast<uintptr_t>(status), a0 = reinterpret_cast<uintptr_t>(a);
      return s0 < a0 + 4 * n && a0 < s0 + sizeof(bitsort_status_t);
    };
    if (n > 0 && (meets(keys) || meets(out))) return BITSORT_ERR_INVALID_ARG;
  }
  Plan p;
  make_plan(n, range_bits, &p);
  if (p.bytes > kNoAllocBytes) return BITSORT_ERR_TOO_LARGE;  // decided before any device call
  void* ws = nullptr;
  if ((rc = noalloc_scratch_of_device(&ws)) != BITSORT_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n == 0) {
    if (status != nullptr)  // a fill kernel, not a memset: the call may be stream-captured
      hipLaunchKernelGGL(serve::k_fill_u64, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned long long*>(status),
                         2u);
    return launch_status();
  }
  static_assert(sizeof(Status) == sizeof(bitsort_status_t), "status layouts must match");
  const bool was = t_capturing;
  t_capturing = true;  // no timing events on this path
  rc = run_plain(p, keys, n, out, ws, s, kEmit, nullptr, nullptr, reinterpret_cast<Status*>(status));
  t_capturing = was;
  return rc;
}

int bitsort_u32(const uint32_t* keys, uint64_t n, uint32_t range_bits, uint32_t* out, bitsort_stream_t stream) {
  int rc = check_args(keys, n, range_bits, out);
  if (rc != BITSORT_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lock(g_mu);
  StreamCtx& c = ctx_for(stream);
  c.used = true;
  if (n == 0) {
    c.last_empty = true;
    return BITSORT_OK;
  }
  Plan p;
  make_plan(n, range_bits, &p);
  rc = grow(&c.ws, &c.bytes, p.bytes, s, c.external);
  if (rc != BITSORT_OK) return rc;
  c.last_empty = false;
  c.last_atomic = false;
  return run_plain(p, keys, n, out, c.ws, s, kEmit, nullptr, nullptr, nullptr, true);
}

int bitsort_u32_atomic(const uint32_t* keys, uint64_t n, uint32_t range_bits, uint32_t* out,
                       bitsort_stream_t stream) {
  int rc = check_args(keys, n, range_bits, out);
  if (rc != BITSORT_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lock(g_mu);
  StreamCtx& c = ctx_for(stream);
  c.used = true;
  if (n == 0) {
    c.last_empty = true;
    return BITSORT_OK;
  }
  if ((rc = init_kernels()) != BITSORT_OK) return rc;
  AtomicPlan p;
  make_atomic_plan(range_bits, &p);
  if (c.atomic_bytes < p.bytes || c.atomic_ws == nullptr) {
    rc = grow(&c.atomic_ws, &c.atomic_bytes, p.bytes, s);
    if (rc != BITSORT_OK) return rc;
    // zero once, when allocated: the bit-vector and the counter are kept zero from here on
    if (hipMemsetAsync(c.atomic_ws, 0, c.atomic_bytes, s) != hipSuccess) return BITSORT_ERR_HIP;
  }
  c.last_empty = false;
  c.last_atomic = true;
  return run_atomic(p, keys, n, range_bits, out, c.atomic_ws, s);
}

size_t bitsort_radix_workspace_bytes(uint64_t n, uint32_t key_bits) {
  if (key_bits > 32 || n > kRadixMaxN) return 0;
  RadixPlan p;
  make_radix_plan(n, key_bits, 4, false, &p);
  return p.bytes;
}

int bitsort_radix_u32_ws(const uint32_t* keys, uint64_t n, uint32_t key_bits, uint32_t* out, void* workspace,
                         size_t ws_bytes, bitsort_stream_t stream) {
  int rc = check_radix_args(keys, n, key_bits, 4, out);
  if (rc != BITSORT_OK) return rc;
  if (workspace == nullptr || (reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return BITSORT_ERR_INVALID_ARG;
  RadixPlan p;
  make_radix_plan(n, key_bits, 4, false, &p);
  if (ws_bytes < p.bytes) return BITSORT_ERR_NO_MEMORY;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n == 0) {  // a zero status through a fill kernel (the call may be stream-captured)
    hipLaunchKernelGGL(serve::k_fill_u64, dim3(1), dim3(64), 0, s, static_cast<unsigned long long*>(workspace), 2u);
    return launch_status();
  }
  if ((rc = init_kernels()) != BITSORT_OK) return rc;
  return run_radix<uint32_t, false>(p, keys, nullptr, n, key_bits, 0u, out, nullptr, workspace, s);
}

int bitsort_count_u32(const uint32_t* keys, uint64_t n, uint32_t range_bits, uint32_t* out, bitsort_stream_t stream) {
  if (range_bits > kCountMaxRangeBits) return BITSORT_ERR_INVALID_ARG;
  if (n > 0 && (keys == nullptr || out == nullptr)) return BITSORT_ERR_INVALID_ARG;
  if (n >= (1ull << 32)) return BITSORT_ERR_TOO_LARGE;
  if (n > 0 && keys != out) {
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(keys), a1 = a0 + 4 * n;
    const uintptr_t b0 = reinterpret_cast<uintptr_t>(out), b1 = b0 + 4 * n;
    if (a0 < b1 && b0 < a1) return BITSORT_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lock(g_mu);
  StreamCtx& c = ctx_for(stream);
  c.used = true;
  if (n == 0) {
    c.last_empty = true;
    return BITSORT_OK;
  }
  Plan p;
  make_count_plan(n, range_bits, &p);
  int rc = grow(&c.ws, &c.bytes, p.bytes, s, c.external);
  if (rc != BITSORT_OK) return rc;
  c.last_empty = false;
  c.last_atomic = false;
  return run_count(p, keys, n, out, c.ws, s);
}

int bitsort_radix_u32(const uint32_t* keys, uint64_t n, uint32_t key_bits, uint32_t* out, bitsort_stream_t stream) {
  return radix_on_stream<uint32_t, false>(keys, nullptr, n, key_bits, 0u, out, nullptr, stream);
}

int bitsort_radix_i32(const int32_t* keys, uint64_t n, int32_t* out, bitsort_stream_t stream) {
  return radix_on_stream<uint32_t, false>(reinterpret_cast<const uint32_t*>(keys), nullptr, n, 32, 0x80000000u,
                                          reinterpret_cast<uint32_t*>(out), nullptr, stream);
}

int bitsort_radix_u64(const uint64_t* keys, uint64_t n, uint32_t key_bits, uint64_t* out, bitsort_stream_t stream) {
  return radix_on_stream<uint64_t, false>(keys, nullptr, n, key_bits, 0ull, out, nullptr, stream);
}

int bitsort_radix_pairs_u32(const uint32_t* keys, const uint32_t* values, uint64_t n, uint32_t key_bits,
                            uint32_t* out_keys, uint32_t* out_values, bitsort_stream_t stream) {
  return radix_on_stream<uint32_t, true>(keys, values, n, key_bits, 0u, out_keys, out_values, stream);
}

constexpr uint32_t kPairsMaxRangeBits = 30;  // the table route: 4 bytes per possible key, at most 4 GiB

// Plan of a key-value sort.  Records route for more than 8192 keys at a
// density above 1/256 (n > 2^range_bits / 256): there it measured faster than
// the table route, whose random stores cost about 76 ps per record against
// the records route's R/32 words of LDS work plus about 10 ps per record.
// Its slice width is the widest of at most 2^18 bits (and at most 4096
// slices) whose expected records fit, with 1/8 to spare, in the LDS that its
// bits and their word prefixes leave; inputs too dense for any take the
// narrowest width and the route's second gather.  Else the table route, over
// the plain plan.
struct PairsPlan {
  bool records = false;
  uint32_t rb = 0, sb = 0, nb = 1, tile_log2 = 0, tile_keys = 0, nt = 0;
  bool short_units = false;
  size_t off_info = 0, off_table = 0, off_stg = 0, bytes = 0;
  Plan plain;                 // table route
  size_t off_vtable = 0;      // table route: the value table, 4 * 2^rb bytes
};

void make_pairs_plan(uint64_t n, uint32_t rb, PairsPlan* p) {
  *p = PairsPlan();
  p->rb = rb;
  const uint32_t lo = std::max(kMinSliceBits, rb > kMaxBucketsLog2 ? rb - kMaxBucketsLog2 : 0u);
  const uint32_t hi = std::min(kPairsMaxSliceBits, rb);
  const bool dense = (n << 8) > (1ull << rb);
  if (n > kDirectMaxN && rb > kMinSliceBits && lo <= hi && dense) {
    uint32_t sb = lo;
    for (uint32_t w = hi; w >= lo; --w) {
      const uint64_t expect = ((n << w) >> rb) + 1u;  // records per slice, uniform keys
      if (expect + expect / 8u <= pairs_record_cap(w)) {
        sb = w;
        break;
      }
    }
    p->records = true;
    p->sb = sb;
    p->nb = 1u << (rb - sb);
    // 2^15-record tiles once there are 2048 slices or more (segments of a
    // few records each otherwise), 2^14 for other large inputs
    p->tile_log2 = n >= (1ull << 22) ? (p->nb >= 2048 ? 15u : 14u) : 12u;
    p->tile_keys = 1u << p->tile_log2;
    p->nt = static_cast<uint32_t>((n + p->tile_keys - 1) >> p->tile_log2);
    p->short_units = (static_cast<uint64_t>(p->tile_keys) << sb) <= (8ull << rb);
    p->off_info = kHeaderBytes;
    p->off_table = align256(p->off_info + 24ull * p->nb);
    p->off_stg = align256(p->off_table + 4ull * p->nt * (p->nb + 1));
    p->bytes = align256(p->off_stg + 8ull * p->nt * p->tile_keys);
    return;
  }
  make_plan(n, rb, &p->plain);
  p->off_vtable = align256(p->plain.bytes);
  p->bytes = p->off_vtable + (4ull << rb);
}

int run_pairs_records(const PairsPlan& p, const uint32_t* keys, const uint32_t* values, uint64_t n,
                      uint32_t* out_keys, uint32_t* out_values, void* ws, hipStream_t stream) {
  char* base = static_cast<char*>(ws);
  Status* status = reinterpret_cast<Status*>(base);
  uint64_t* info = reinterpret_cast<uint64_t*>(base + p.off_info);
  uint32_t* table = reinterpret_cast<uint32_t*>(base + p.off_table);
  uint32_t* stg = reinterpret_cast<uint32_t*>(base + p.off_stg);
  const uint64_t range = 1ull << p.rb;
  const int vec_ok = ((reinterpret_cast<uintptr_t>(keys) | reinterpret_cast<uintptr_t>(values)) % 16u) == 0 ? 1 : 0;
  const size_t part_lds = 4ull * (32 + round_up4(p.nb) + p.tile_keys);
  const uint32_t grid = 8u * ((p.nt + 7u) / 8u);  // the 8-way XCD mapping of tiles
  int rc;
  {
    LaunchTimer timer(kKPartitionKV, stream);
    if (p.tile_log2 == 12)
      hipLaunchKernelGGL((k_partition_kv<1024, 4>), dim3(grid), dim3(1024), part_lds, stream, keys, values, n, range,
                         p.sb, p.nb, p.nt, stg, table, vec_ok);
    else if (p.tile_log2 == 14)
      hipLaunchKernelGGL((k_partition_kv<1024, 16>), dim3(grid), dim3(1024), part_lds, stream, keys, values, n,
                         range, p.sb, p.nb, p.nt, stg, table, vec_ok);
    else
      hipLaunchKernelGGL((k_partition_kv<1024, 32>), dim3(grid), dim3(1024), part_lds, stream, keys, values, n,
                         range, p.sb, p.nb, p.nt, stg, table, vec_ok);
    if ((rc = launch_status()) != BITSORT_OK) return rc;
  }
  {
    LaunchTimer timer(kKSliceKV, stream);
    auto kernel = p.short_units ? k_slice_kv<kSliceBlock, kSliceUnroll, 16> : k_slice_kv<kSliceBlock, kSliceUnroll, 64>;
    hipLaunchKernelGGL(kernel, dim3(8u * ((p.nb + 7u) / 8u)), dim3(kSliceBlock), kLdsBytes, stream,
                       reinterpret_cast<const uint2*>(stg), table, p.nt, p.tile_keys, p.sb, p.nb, out_keys, out_values, info);
    if ((rc = launch_status()) != BITSORT_OK) return rc;
  }
  LaunchTimer timer(kKPairsFinish, stream);
  hipLaunchKernelGGL((k_pairs_finish<kSliceBlock>), dim3(1), dim3(kSliceBlock), 0, stream, n, p.nb, info, status,
                     out_keys, out_values);
  return launch_status();
}

int run_pairs_table(const PairsPlan& p, const uint32_t* keys, const uint32_t* values, uint64_t n,
                    uint32_t* out_keys, uint32_t* out_values, void* ws, hipStream_t stream) {
  uint32_t* table = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + p.off_vtable);
  const uint64_t range = 1ull << p.rb;
  const dim3 grid(static_cast<uint32_t>((n + kPairsPerBlock - 1) / kPairsPerBlock));
  int rc;
  {
    // before the sort, which may write over keys (out_keys == keys)
    LaunchTimer timer(kKPairsScatter, stream);
    hipLaunchKernelGGL(k_pairs_scatter, grid, dim3(kPairsBlock), 0, stream, keys, values, n, range, table);
    if ((rc = launch_status()) != BITSORT_OK) return rc;
  }
  // the finish step in the stream: a repeated key's compaction comes before the gather
  if ((rc = run_plain(p.plain, keys, n, out_keys, ws, stream, kEmit, nullptr, nullptr, nullptr, false)) != BITSORT_OK)
    return rc;
  LaunchTimer timer(kKPairsGather, stream);
  hipLaunchKernelGGL(k_pairs_gather, grid, dim3(kPairsBlock), 0, stream, out_keys, n, range, table, out_values);
  return launch_status();
}

int bitsort_pairs_u32(const uint32_t* keys, const uint32_t* values, uint64_t n, uint32_t range_bits,
                      uint32_t* out_keys, uint32_t* out_values, bitsort_stream_t stream) {
  int rc = check_args(keys, n, range_bits, out_keys);
  if (rc != BITSORT_OK) return rc;
  if (range_bits > kPairsMaxRangeBits) return BITSORT_ERR_INVALID_ARG;
  if (n > 0) {
    if (values == nullptr || out_values == nullptr) return BITSORT_ERR_INVALID_ARG;
    auto meets = [&](const void* a, const void* b) {  // [a, a + 4n) against [b, b + 4n)
      const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
      return a0 < b0 + 4 * n && b0 < a0 + 4 * n;
    };
    if (values != out_values && meets(values, out_values)) return BITSORT_ERR_INVALID_ARG;
    for (const void* k : {static_cast<const void*>(keys), static_cast<const void*>(out_keys)})
      for (const void* v : {static_cast<const void*>(values), static_cast<const void*>(out_values)})
        if (meets(k, v)) return BITSORT_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lock(g_mu);
  StreamCtx& c = ctx_for(stream);
  c.used = true;
  if (n == 0) {
    c.last_empty = true;
    return BITSORT_OK;
  }
  if ((rc = init_kernels()) != BITSORT_OK) return rc;
  PairsPlan p;
  make_pairs_plan(n, range_bits, &p);
  rc = grow(&c.ws, &c.bytes, p.bytes, s, c.external);
  if (rc != BITSORT_OK) return rc;
  c.last_empty = false;
  c.last_atomic = false;
  return p.records ? run_pairs_records(p, keys, values, n, out_keys, out_values, c.ws, s)
                   : run_pairs_table(p, keys, values, n, out_keys, out_values, c.ws, s);
}

int bitsort_i32(const int32_t* keys_s, uint64_t n, uint32_t range_bits, int32_t* out_s, bitsort_stream_t stream) {
  const uint32_t* keys = reinterpret_cast<const uint32_t*>(keys_s);
  uint32_t* out = reinterpret_cast<uint32_t*>(out_s);
  int rc = check_args(keys, n, range_bits, out);
  if (rc != BITSORT_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lock(g_mu);
  StreamCtx& c = ctx_for(stream);
  c.used = true;
  if (n == 0) {
    c.last_empty = true;
    return BITSORT_OK;
  }
  Plan p;
  make_plan(n, range_bits, &p);
  p.bias = range_bits ? (1u << (range_bits - 1)) : 0u;
  rc = grow(&c.ws, &c.bytes, p.bytes, s, c.external);
  if (rc != BITSORT_OK) return rc;
  c.last_empty = false;
  c.last_atomic = false;
  return run_plain(p, keys, n, out, c.ws, s, kEmit, nullptr, nullptr, nullptr, true);
}

int bitsort_get_status(bitsort_stream_t stream, bitsort_status_t* status) {
  if (status == nullptr) return BITSORT_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    StreamCtx& c = ctx_for(stream);
    if (!c.used) return BITSORT_ERR_INVALID_ARG;
    if (c.last_empty) {
      if (hipStreamSynchronize(s) != hipSuccess) return BITSORT_ERR_HIP;
      *status = bitsort_status_t{0, 0, 0};
      return BITSORT_OK;
    }
    ws = c.last_atomic ? c.atomic_ws : c.ws;
  }
  return read_plain_status(ws, s, status);
}

int bitsort_workspace_status(const void* workspace, bitsort_stream_t stream, bitsort_status_t* status) {
  if (workspace == nullptr || status == nullptr) return BITSORT_ERR_INVALID_ARG;
  return read_plain_status(const_cast<void*>(workspace), static_cast<hipStream_t>(stream), status);
}

int bitsort_generate_u32(uint32_t* out, uint64_t first, uint64_t count, uint32_t range_bits, uint64_t seed,
                         bitsort_stream_t stream) {
  if (range_bits > 32 || (count > 0 && out == nullptr)) return BITSORT_ERR_INVALID_ARG;
  if (first + count > (1ull << range_bits) || first + count < first) return BITSORT_ERR_TOO_LARGE;
  if (count == 0) return BITSORT_OK;
  uint32_t k[4];
  splitmix_keys(seed, k);
  const uint64_t blocks = (count + kGenChunk - 1) / kGenChunk;  // count <= 2^32: at most 2^20 blocks
  hipLaunchKernelGGL(k_generate, dim3(static_cast<uint32_t>(blocks)), dim3(kGenBlock), 0,
                     static_cast<hipStream_t>(stream), out, first, count, range_bits, k[0], k[1], k[2], k[3]);
  return launch_status();
}

static int debug_run(const uint32_t* keys, uint64_t n, uint32_t range_bits, int mode, uint32_t* bm,
                     uint64_t* pre, bitsort_stream_t stream) {
  if (range_bits > 30 || (n > 0 && keys == nullptr)) return BITSORT_ERR_INVALID_ARG;
  if (mode == kDumpBitmap && bm == nullptr) return BITSORT_ERR_INVALID_ARG;
  if (mode == kDumpPrefix && pre == nullptr) return BITSORT_ERR_INVALID_ARG;
  if (n > (1ull << range_bits)) return BITSORT_ERR_TOO_LARGE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Plan p;
  make_plan(n, range_bits, &p);
  void* ws = nullptr;
  if (hipMalloc(&ws, p.bytes) != hipSuccess) return BITSORT_ERR_NO_MEMORY;
  int rc = run_plain(p, keys, n, nullptr, ws, s, mode, bm, pre);
  if (hipStreamSynchronize(s) != hipSuccess && rc == BITSORT_OK) rc = BITSORT_ERR_HIP;
  (void)hipFree(ws);
  return rc;
}

int bitsort_debug_bitmap_u32(const uint32_t* keys, uint64_t n, uint32_t range_bits, uint32_t* bitmap,
                             bitsort_stream_t stream) {
  return debug_run(keys, n, range_bits, kDumpBitmap, bitmap, nullptr, stream);
}

int bitsort_debug_prefix_u32(const uint32_t* keys, uint64_t n, uint32_t range_bits, uint64_t* prefix,
                             bitsort_stream_t stream) {
  return debug_run(keys, n, range_bits, kDumpPrefix, nullptr, prefix, stream);
}

int bitsort_batch_u32(const uint32_t* keys, const uint64_t* offsets, uint32_t num_segments,
                      const uint8_t* range_bits, uint32_t* out, uint64_t max_keys, bitsort_stream_t stream) {
  int rc = check_batch_args(keys, offsets, num_segments, range_bits, out, max_keys);
  if (rc != BITSORT_OK) return rc;
  rc = init_kernels();
  if (rc != BITSORT_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const BatchTuning t = batch_tuning();
  const size_t bytes = batch_workspace_bytes(num_segments, t);
  std::lock_guard<std::mutex> lock(g_mu);
  StreamCtx& c = ctx_for(stream);
  rc = grow(&c.batch_ws, &c.batch_bytes, bytes, s);
  if (rc != BITSORT_OK) return rc;
  c.batch_segments = num_segments;
  return run_batch(keys, offsets, num_segments, range_bits, out, max_keys, c.batch_ws, s, t);
}

int bitsort_batch_ptr_u32(const uint32_t* const* keys, const uint64_t* n, const uint8_t* range_bits,
                          uint32_t* const* out, uint32_t count, bitsort_stream_t stream) {
  int rc = check_multi_args(keys, n, range_bits, out, count);
  if (rc != BITSORT_OK) return rc;
  MultiPlan p;
  if ((rc = make_multi_plan(keys, n, range_bits, out, count, &p)) != BITSORT_OK) return rc;
  std::lock_guard<std::mutex> lock(g_mu);
  StreamCtx& c = ctx_for(stream);
  return multi_on_stream(c, p, count, static_cast<hipStream_t>(stream));
}

int bitsort_u64(const uint64_t* keys, uint64_t n, uint32_t range_bits, uint64_t* out, bitsort_stream_t stream) {
  if (range_bits > kWideMaxRangeBits) return BITSORT_ERR_INVALID_ARG;
  if (n > 0 && (keys == nullptr || out == nullptr)) return BITSORT_ERR_INVALID_ARG;
  if (n >= (1ull << 32) || n > (1ull << range_bits)) return BITSORT_ERR_TOO_LARGE;
  if (n > 0 && static_cast<const void*>(keys) != static_cast<const void*>(out) && overlaps(keys, out, 8 * n))
    return BITSORT_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lock(g_mu);
  StreamCtx& c = ctx_for(stream);
  c.used = true;
  if (n == 0) {
    c.last_empty = true;
    return BITSORT_OK;
  }
  int rc = init_kernels();
  if (rc != BITSORT_OK) return rc;
  c.last_empty = false;
  c.last_atomic = false;
  return run_wide(c, keys, n, range_bits, out, s);
}

int bitsort_batch_status(bitsort_stream_t stream, bitsort_status_t* status, uint32_t num_segments) {
  if (status == nullptr) return BITSORT_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    StreamCtx& c = ctx_for(stream);
    if (c.batch_ws == nullptr || num_segments > c.batch_segments) return BITSORT_ERR_INVALID_ARG;
    ws = c.batch_ws;
  }
  if (hipStreamSynchronize(s) != hipSuccess) return BITSORT_ERR_HIP;
  static_assert(sizeof(SegStatus) == sizeof(bitsort_status_t), "status layouts must match");
  if (num_segments == 0) return BITSORT_OK;
  if (hipMemcpy(status, static_cast<char*>(ws) + kHeaderBytes, sizeof(SegStatus) * num_segments,
                hipMemcpyDeviceToHost) != hipSuccess)
    return BITSORT_ERR_HIP;
  return BITSORT_OK;
}

int bitsort_set_workspace(void* workspace, size_t bytes, bitsort_stream_t stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (workspace != nullptr && ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0 || bytes < kHeaderBytes))
    return BITSORT_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_mu);
  StreamCtx& c = ctx_for(stream);
  if (c.ws != nullptr && !c.external) {  // the library's own allocation goes; earlier work on it must end first
    if (hipStreamSynchronize(s) != hipSuccess || hipFree(c.ws) != hipSuccess) return BITSORT_ERR_HIP;
  }
  c.ws = workspace;
  c.bytes = workspace != nullptr ? bytes : 0;
  c.external = workspace != nullptr;
  c.last_empty = true;  // the status of a call made before now is gone with the old workspace
  return BITSORT_OK;
}

// ---- batch plans: host-checked segments, workspace fixed up front --------------

struct bitsort_batch_plan {
  void* ws = nullptr;
  size_t ws_bytes = 0;
  uint32_t segments = 0;
  uint64_t max_keys = 0;
  BatchTuning tuning;
  int device = 0;
};

int bitsort_batch_plan(const uint64_t* offsets, const uint8_t* range_bits, uint32_t num_segments,
                       bitsort_batch_plan_t** plan) {
  if (plan == nullptr) return BITSORT_ERR_INVALID_ARG;
  *plan = nullptr;
  if (offsets == nullptr || range_bits == nullptr || num_segments == 0 || num_segments > BITSORT_BATCH_MAX_SEGMENTS)
    return BITSORT_ERR_INVALID_ARG;
  if (offsets[0] != 0) return BITSORT_ERR_INVALID_ARG;
  for (uint32_t i = 0; i < num_segments; ++i) {
    if (range_bits[i] > kMaxBatchRangeBits || offsets[i + 1] < offsets[i]) return BITSORT_ERR_INVALID_ARG;
    if (offsets[i + 1] - offsets[i] > (1ull << range_bits[i])) return BITSORT_ERR_TOO_LARGE;
  }
  if (offsets[num_segments] >= (1ull << 40)) return BITSORT_ERR_TOO_LARGE;
  int rc = init_kernels();
  if (rc != BITSORT_OK) return rc;
  auto* p = new struct bitsort_batch_plan();
  p->segments = num_segments;
  p->max_keys = offsets[num_segments];
  p->tuning = batch_tuning();
  p->ws_bytes = batch_workspace_bytes(num_segments, p->tuning);
  (void)hipGetDevice(&p->device);
  if (hipMalloc(&p->ws, p->ws_bytes) != hipSuccess) {
    (void)hipGetLastError();
    delete p;
    return BITSORT_ERR_NO_MEMORY;
  }
  *plan = p;
  return BITSORT_OK;
}

int bitsort_batch_run(const bitsort_batch_plan_t* plan, const uint32_t* keys, const uint64_t* offsets,
                      const uint8_t* range_bits, uint32_t* out, bitsort_stream_t stream) {
  if (plan == nullptr) return BITSORT_ERR_INVALID_ARG;
  int rc = check_batch_args(keys, offsets, plan->segments, range_bits, out, plan->max_keys);
  if (rc != BITSORT_OK) return rc;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != plan->device) return BITSORT_ERR_INVALID_ARG;
  return run_batch(keys, offsets, plan->segments, range_bits, out, plan->max_keys, plan->ws,
                   static_cast<hipStream_t>(stream), plan->tuning);
}

int bitsort_batch_plan_status(const bitsort_batch_plan_t* plan, bitsort_stream_t stream, bitsort_status_t* status,
                              uint32_t count) {
  if (plan == nullptr || status == nullptr || count > plan->segments) return BITSORT_ERR_INVALID_ARG;
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return BITSORT_ERR_HIP;
  if (count == 0) return BITSORT_OK;
  if (hipMemcpy(status, static_cast<const char*>(plan->ws) + kHeaderBytes, sizeof(SegStatus) * count,
                hipMemcpyDeviceToHost) != hipSuccess)
    return BITSORT_ERR_HIP;
  return BITSORT_OK;
}

int bitsort_batch_plan_destroy(bitsort_batch_plan_t* plan) {
  if (plan == nullptr) return BITSORT_OK;
  const int rc = (plan->ws != nullptr && hipFree(plan->ws) != hipSuccess) ? BITSORT_ERR_HIP : BITSORT_OK;
  delete plan;
  return rc;
}

// ---- graphs -------------------------------------------------------------------

struct bitsort_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* ws = nullptr;
  bool batch = false;
  uint32_t segments = 0;
  int device = 0;
};

static int capture(bitsort_graph* g, const std::function<int(hipStream_t)>& enqueue) {
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return BITSORT_ERR_HIP;
  int rc = BITSORT_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    rc = BITSORT_ERR_HIP;
  } else {
    t_capturing = true;
    rc = enqueue(cs);
    t_capturing = false;
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &graph);
    if (rc == BITSORT_OK && e != hipSuccess) rc = BITSORT_ERR_HIP;
    if (rc == BITSORT_OK) {
      g->graph = graph;
      if (hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) rc = BITSORT_ERR_HIP;
    } else if (graph != nullptr) {
      (void)hipGraphDestroy(graph);
    }
  }
  (void)hipStreamDestroy(cs);
  return rc;
}

int bitsort_graph_create_u32(const uint32_t* keys, uint64_t n, uint32_t range_bits, uint32_t* out,
                             bitsort_graph_t** graph) {
  if (graph == nullptr) return BITSORT_ERR_INVALID_ARG;
  *graph = nullptr;
  int rc = check_args(keys, n, range_bits, out);
  if (rc != BITSORT_OK) return rc;
  if (n == 0) return BITSORT_ERR_INVALID_ARG;
  rc = init_kernels();
  if (rc != BITSORT_OK) return rc;
  Plan p;
  make_plan(n, range_bits, &p);
  auto* g = new bitsort_graph();
  (void)hipGetDevice(&g->device);
  if (hipMalloc(&g->ws, p.bytes) != hipSuccess) {
    delete g;
    return BITSORT_ERR_NO_MEMORY;
  }
  rc = capture(g, [&](hipStream_t cs) {
    return run_plain(p, keys, n, out, g->ws, cs, kEmit, nullptr, nullptr, nullptr, true);
  });
  if (rc != BITSORT_OK) {
    bitsort_graph_destroy(g);
    return rc;
  }
  *graph = g;
  return BITSORT_OK;
}

int bitsort_graph_create_batch_u32(const uint32_t* keys, const uint64_t* offsets, uint32_t num_segments,
                                   const uint8_t* range_bits, uint32_t* out, uint64_t max_keys,
                                   bitsort_graph_t** graph) {
  if (graph == nullptr) return BITSORT_ERR_INVALID_ARG;
  *graph = nullptr;
  int rc = check_batch_args(keys, offsets, num_segments, range_bits, out, max_keys);
  if (rc != BITSORT_OK) return rc;
  rc = init_kernels();
  if (rc != BITSORT_OK) return rc;
  const BatchTuning t = batch_tuning();
  auto* g = new bitsort_graph();
  g->batch = true;
  g->segments = num_segments;
  (void)hipGetDevice(&g->device);
  if (hipMalloc(&g->ws, batch_workspace_bytes(num_segments, t)) != hipSuccess) {
    delete g;
    return BITSORT_ERR_NO_MEMORY;
  }
  rc = capture(g, [&](hipStream_t cs) {
    return run_batch(keys, offsets, num_segments, range_bits, out, max_keys, g->ws, cs, t);
  });
  if (rc != BITSORT_OK) {
    bitsort_graph_destroy(g);
    return rc;
  }
  *graph = g;
  return BITSORT_OK;
}

int bitsort_graph_launch(bitsort_graph_t* graph, bitsort_stream_t stream) {
  if (graph == nullptr || graph->exec == nullptr) return BITSORT_ERR_INVALID_ARG;
  return hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream)) == hipSuccess ? BITSORT_OK : BITSORT_ERR_HIP;
}

int bitsort_graph_status(bitsort_graph_t* graph, bitsort_stream_t stream, bitsort_status_t* status,
                         uint32_t count) {
  if (graph == nullptr || status == nullptr) return BITSORT_ERR_INVALID_ARG;
  if (count > (graph->batch ? graph->segments : 1u)) return BITSORT_ERR_INVALID_ARG;
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return BITSORT_ERR_HIP;
  if (count == 0) return BITSORT_OK;
  if (!graph->batch) return read_plain_status(graph->ws, static_cast<hipStream_t>(stream), status);
  const char* src = static_cast<const char*>(graph->ws) + kHeaderBytes;
  static_assert(sizeof(Status) == sizeof(bitsort_status_t), "status layouts must match");
  if (hipMemcpy(status, src, sizeof(bitsort_status_t) * count, hipMemcpyDeviceToHost) != hipSuccess)
    return BITSORT_ERR_HIP;
  return BITSORT_OK;
}

int bitsort_graph_destroy(bitsort_graph_t* graph) {
  if (graph == nullptr) return BITSORT_OK;
  int rc = BITSORT_OK;
  if (graph->exec && hipGraphExecDestroy(graph->exec) != hipSuccess) rc = BITSORT_ERR_HIP;
  if (graph->graph && hipGraphDestroy(graph->graph) != hipSuccess) rc = BITSORT_ERR_HIP;
  if (graph->ws && hipFree(graph->ws) != hipSuccess) rc = BITSORT_ERR_HIP;
  delete graph;
  return rc;
}

// ---- autotuning -----------------------------------------------------------------

static float time_ms(const std::function<int()>& run, int reps, hipStream_t s, int* rc) {
  hipEvent_t a = nullptr, b = nullptr;
  float ms = -1.f;
  *rc = BITSORT_OK;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    *rc = BITSORT_ERR_HIP;
  } else {
    *rc = run();  // warm-up (also grows workspaces)
    if (*rc == BITSORT_OK && hipEventRecord(a, s) == hipSuccess) {
      for (int r = 0; r < reps && *rc == BITSORT_OK; ++r) *rc = run();
      if (*rc == BITSORT_OK && hipEventRecord(b, s) == hipSuccess && hipEventSynchronize(b) == hipSuccess &&
          hipEventElapsedTime(&ms, a, b) == hipSuccess)
        ms /= static_cast<float>(reps);
      else if (*rc == BITSORT_OK)
        *rc = BITSORT_ERR_HIP;
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  return ms;
}

int bitsort_autotune_u32(uint64_t n, uint32_t range_bits, int reps, bitsort_stream_t stream,
                         bitsort_tuning_t* best) {
  if (best == nullptr || reps < 1 || range_bits > 32 || n == 0 || n > (1ull << range_bits) || n >= (1ull << 32))
    return BITSORT_ERR_INVALID_ARG;
  int rc = init_kernels();
  if (rc != BITSORT_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Plan base_plan;
  make_plan(n, range_bits, &base_plan);
  *best = bitsort_tuning_t{};
  if (base_plan.direct) return BITSORT_OK;  // nothing to choose
  uint32_t *keys = nullptr, *out = nullptr;
  if (hipMalloc(&keys, 4 * n) != hipSuccess) return BITSORT_ERR_NO_MEMORY;
  if (hipMalloc(&out, 4 * n) != hipSuccess) {
    (void)hipFree(keys);
    return BITSORT_ERR_NO_MEMORY;
  }
  rc = bitsort_generate_u32(keys, 0, n, range_bits, 0x5EEDull + range_bits, stream);
  // Candidates: the five widest slice sizes the fan-out limit allows, every
  // tile size, every emit path (the summary one only where it applies).
  const uint32_t sb_lo = std::max<uint32_t>(kMinSliceBits, range_bits > kMaxBucketsLog2 ? range_bits - kMaxBucketsLog2 : 0);
  const uint32_t sb_hi = std::min(kMaxSliceBits, range_bits);
  void* ws = nullptr;
  size_t ws_bytes = 0;
  float best_ms = 1e30f;
  for (uint32_t sb = std::max(sb_lo, sb_hi >= 4 ? sb_hi - 4 : 0); sb <= sb_hi && rc == BITSORT_OK; ++sb) {
    for (uint32_t tl = 12; tl <= 15 && rc == BITSORT_OK; ++tl) {
      for (uint32_t path = 1; path <= 3 && rc == BITSORT_OK; ++path) {
        const PlainTuning cand{sb, tl, path, 0.f};
        Plan p;
        make_plan(n, range_bits, &p, &cand);
        if (p.direct || p.sb != sb || p.tile_log2 != tl || (path == 2) != p.via_bitvec || (path == 3) != p.sparse)
          continue;
        rc = grow(&ws, &ws_bytes, p.bytes, s);
        if (rc != BITSORT_OK) break;
        const float ms = time_ms([&] { return run_plain(p, keys, n, out, ws, s, kEmit, nullptr, nullptr, nullptr, true); },
                                 reps, s, &rc);
        if (rc == BITSORT_OK && ms >= 0.f && ms < best_ms) {
          best_ms = ms;
          *best = bitsort_tuning_t{sb, tl, path, 0, ms};
        }
      }
    }
  }
  (void)hipStreamSynchronize(s);
  if (ws) (void)hipFree(ws);
  (void)hipFree(keys);
  (void)hipFree(out);
  if (rc == BITSORT_OK && best->slice_bits != 0) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_plain_tuned[{range_bits, ceil_log2(n)}] = PlainTuning{best->slice_bits, best->tile_log2, best->emit_path, best->ms};
  }
  return rc;
}

int bitsort_autotune_batch_u32(const uint32_t* keys, const uint64_t* offsets, uint32_t num_segments,
                               const uint8_t* range_bits, uint32_t* out, uint64_t max_keys, int reps,
                               bitsort_stream_t stream, bitsort_tuning_t* best) {
  if (best == nullptr || reps < 1) return BITSORT_ERR_INVALID_ARG;
  int rc = check_batch_args(keys, offsets, num_segments, range_bits, out, max_keys);
  if (rc != BITSORT_OK) return rc;
  rc = init_kernels();
  if (rc != BITSORT_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  *best = bitsort_tuning_t{};
  float best_ms = 1e30f;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  for (uint32_t block : {256u, 512u, 1024u}) {
    for (uint32_t sbb = 16; sbb <= kBatchSliceBits && rc == BITSORT_OK; ++sbb) {
      const BatchTuning t{block, sbb};
      rc = grow(&ws, &ws_bytes, batch_workspace_bytes(num_segments, t), s);
      if (rc != BITSORT_OK) break;
      const float ms = time_ms([&] {
        return run_batch(keys, offsets, num_segments, range_bits, out, max_keys, ws, s, t);
      }, reps, s, &rc);
      if (rc == BITSORT_OK && ms >= 0.f && ms < best_ms) {
        best_ms = ms;
        *best = bitsort_tuning_t{sbb, 0, 0, block, ms};
      }
    }
  }
  (void)hipStreamSynchronize(s);
  if (ws) (void)hipFree(ws);
  if (rc == BITSORT_OK && best->batch_block != 0) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_batch_tuned = BatchTuning{best->batch_block, best->slice_bits};
  }
  return rc;
}

static std::string device_key() {
  int dev = 0, cus = 0;
  hipDeviceProp_t prop{};
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
  }
  return arch + ":" + std::to_string(cus);
}

int bitsort_tuning_save(const char* path) {
  if (path == nullptr) return BITSORT_ERR_INVALID_ARG;
  FILE* f = std::fopen(path, "w");
  if (f == nullptr) return BITSORT_ERR_INVALID_ARG;
  const std::string dk = device_key();
  std::lock_guard<std::mutex> lock(g_tune_mu);
  for (const auto& kv : g_plain_tuned)
    std::fprintf(f, "{\"device\": \"%s\", \"kind\": \"plain\", \"range_bits\": %u, \"log2n\": %u, "
                    "\"slice_bits\": %u, \"tile_log2\": %u, \"emit_path\": %u, \"ms\": %.5f}\n",
                 dk.c_str(), kv.first.first, kv.first.second, kv.second.slice_bits, kv.second.tile_log2,
                 kv.second.emit_path, kv.second.ms);
  std::fprintf(f, "{\"device\": \"%s\", \"kind\": \"batch\", \"block\": %u, \"slice_bits\": %u}\n", dk.c_str(),
               g_batch_tuned.block, g_batch_tuned.slice_bits);
  return std::fclose(f) == 0 ? BITSORT_OK : BITSORT_ERR_INVALID_ARG;
}

int bitsort_tuning_load(const char* path, int* entries) {
  if (path == nullptr) return BITSORT_ERR_INVALID_ARG;
  FILE* f = std::fopen(path, "r");
  if (f == nullptr) return BITSORT_ERR_INVALID_ARG;
  const std::string dk = device_key();
  char line[512], dev[128];
  int count = 0;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  while (std::fgets(line, sizeof line, f)) {
    unsigned rb, l2, sb, tl, ep, block;
    float ms;
    if (std::sscanf(line, "{\"device\": \"%127[^\"]\", \"kind\": \"plain\", \"range_bits\": %u, \"log2n\": %u, "
                          "\"slice_bits\": %u, \"tile_log2\": %u, \"emit_path\": %u, \"ms\": %f}",
                    dev, &rb, &l2, &sb, &tl, &ep, &ms) == 7) {
      if (dk != dev || rb > 32 || sb < kMinSliceBits || sb > kMaxSliceBits || tl < 12 || tl > 15 || ep > 4) continue;
      g_plain_tuned[{rb, l2}] = PlainTuning{sb, tl, ep, ms};
      ++count;
    } else if (std::sscanf(line, "{\"device\": \"%127[^\"]\", \"kind\": \"batch\", \"block\": %u, \"slice_bits\": %u}",
                           dev, &block, &sb) == 3) {
      if (dk != dev || (block != 256 && block != 512 && block != 1024) || sb < 16 || sb > kBatchSliceBits) continue;
      g_batch_tuned = BatchTuning{block, sb};
      ++count;
    }
  }
  std::fclose(f);
  if (entries) *entries = count;
  return BITSORT_OK;
}

int bitsort_tuning_clear(void) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_plain_tuned.clear();
  g_batch_tuned = BatchTuning{};
  return BITSORT_OK;
}

int bitsort_serve_run(const bitsort_request_t* requests, uint32_t count, const bitsort_serve_config_t* config,
                      bitsort_request_result_t* results, bitsort_serve_stats_t* stats) {
  if (config == nullptr || (count > 0 && (requests == nullptr || results == nullptr))) return BITSORT_ERR_INVALID_ARG;
  const bitsort_serve_config_t& c = *config;
  if (c.streams < 1 || c.streams > 16 || c.max_batch_requests < 1 || c.max_batch_keys < 1 || c.budget_bytes == 0)
    return BITSORT_ERR_INVALID_ARG;
  if (c.simulate && !(c.sim_keys_per_s > 0.0 && c.sim_overhead_s >= 0.0)) return BITSORT_ERR_INVALID_ARG;
  if (c.max_batch_requests > BITSORT_BATCH_MAX_SEGMENTS) return BITSORT_ERR_INVALID_ARG;
  serve::Arena arena;
  arena.init(c.budget_bytes);
  if (c.simulate) {
    serve::SimExecutor ex(c.sim_overhead_s, c.sim_keys_per_s);
    return serve::schedule(ex, arena, requests, count, c, results, stats, true);
  }
  if (reinterpret_cast<uintptr_t>(c.arena) % 256 != 0) return BITSORT_ERR_INVALID_ARG;
  int rc = init_kernels();
  if (rc != BITSORT_OK) return rc;
  void* base = c.arena;
  if (base == nullptr && hipMalloc(&base, c.budget_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return BITSORT_ERR_NO_MEMORY;
  }
  {
    serve::HipExecutor ex;  // its destructor waits for every slot stream
    rc = ex.init(static_cast<char*>(base), c.streams, c.verify != 0, c.max_batch_requests, c.outputs);
    if (rc == BITSORT_OK) rc = serve::schedule(ex, arena, requests, count, c, results, stats, false);
  }
  if (c.arena == nullptr) {
    (void)hipDeviceSynchronize();
    (void)hipFree(base);
  }
  return rc;
}

int bitsort_digest_u32(const uint32_t* data, uint64_t n, uint64_t* digest, bitsort_stream_t stream) {
  if (digest == nullptr || (n > 0 && data == nullptr)) return BITSORT_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint64_t* dev = nullptr;
  if (hipMalloc(&dev, 64) != hipSuccess) return BITSORT_ERR_NO_MEMORY;
  const uint64_t hoff[2] = {0, n};
  int rc = BITSORT_OK;
  if (hipMemcpyAsync(dev + 1, hoff, 16, hipMemcpyHostToDevice, s) != hipSuccess) rc = BITSORT_ERR_HIP;
  if (rc == BITSORT_OK) {
    hipLaunchKernelGGL(serve::k_fill_u64, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned long long*>(dev), 1u);
    if (n > 0)
      hipLaunchKernelGGL(serve::k_digest, dim3(static_cast<uint32_t>((n + serve::kDigestChunk - 1) / serve::kDigestChunk)),
                         dim3(256), 0, s, data, dev + 1, 1u, n, reinterpret_cast<unsigned long long*>(dev));
    rc = launch_status();
  }
  if (rc == BITSORT_OK && (hipMemcpyAsync(digest, dev, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
                           hipStreamSynchronize(s) != hipSuccess))
    rc = BITSORT_ERR_HIP;
  (void)hipFree(dev);
  return rc;
}


int bitsort_profile_enable(int on) {
  g_prof_on.store(on != 0);
  return BITSORT_OK;
}

int bitsort_profile_reset(void) {
  std::lock_guard<std::mutex> lock(g_prof_mu);
  for (auto& t : g_prof_pending) {
    (void)hipEventSynchronize(t.stop);
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  g_prof_pending.clear();
  for (int k = 0; k < kKCount; ++k) {
    g_prof_launches[k] = 0;
    g_prof_ms[k] = 0.0;
  }
  return BITSORT_OK;
}

int bitsort_profile_read(bitsort_profile_entry_t* entries, int max_entries, int* n_entries) {
  if (n_entries == nullptr || (max_entries > 0 && entries == nullptr)) return BITSORT_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_prof_mu);
  int rc = BITSORT_OK;
  for (auto& t : g_prof_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(t.stop) != hipSuccess || hipEventElapsedTime(&ms, t.start, t.stop) != hipSuccess)
      rc = BITSORT_ERR_HIP;
    g_prof_launches[t.kernel] += 1;
    g_prof_ms[t.kernel] += ms;
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  g_prof_pending.clear();
  int n = 0;
  for (int k = 0; k < kKCount; ++k) {
    if (g_prof_launches[k] == 0) continue;
    if (n < max_entries) {
      std::memset(entries[n].kernel, 0, sizeof(entries[n].kernel));
      std::strncpy(entries[n].kernel, kKernelNames[k], sizeof(entries[n].kernel) - 1);
      entries[n].launches = g_prof_launches[k];
      entries[n].total_ms = g_prof_ms[k];
    }
    ++n;
  }
  *n_entries = n;
  return rc;
}

int bitsort_set_tuning(uint32_t slice_bits, uint32_t tile_log2, uint32_t emit_path) {
  if (slice_bits != 0 && (slice_bits < kMinSliceBits || slice_bits > kMaxSliceBits)) return BITSORT_ERR_INVALID_ARG;
  if (tile_log2 != 0 && (tile_log2 < 12 || tile_log2 > 15)) return BITSORT_ERR_INVALID_ARG;
  if (emit_path > 4) return BITSORT_ERR_INVALID_ARG;
  g_tune_sb.store(slice_bits);
  g_tune_tile.store(tile_log2);
  g_tune_path.store(emit_path);
  return BITSORT_OK;
}

int bitsort_debug_split_u32(const void* workspace, uint64_t n, uint32_t range_bits, uint32_t* published,
                            bitsort_stream_t stream) {
  if (workspace == nullptr || published == nullptr || range_bits > 32) return BITSORT_ERR_INVALID_ARG;
  *published = 0;
  Plan p;
  make_plan(n, range_bits, &p);
  if (p.direct || !p.split) return BITSORT_OK;
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return BITSORT_ERR_HIP;
  const char* ctl = static_cast<const char*>(workspace) + p.off_split_ctl;
  return hipMemcpy(published, ctl, sizeof(uint32_t), hipMemcpyDeviceToHost) == hipSuccess ? BITSORT_OK
                                                                                        : BITSORT_ERR_HIP;
}

int bitsort_plan_info(uint64_t n, uint32_t range_bits, uint32_t* slice_bits, uint32_t* tile_log2,
                      uint32_t* buckets, uint32_t* emit_path) {
  if (range_bits > 32 || slice_bits == nullptr || tile_log2 == nullptr || buckets == nullptr ||
      emit_path == nullptr)
    return BITSORT_ERR_INVALID_ARG;
  Plan p;
  make_plan(n, range_bits, &p);
  *slice_bits = p.sb;
  *tile_log2 = p.direct ? 0 : p.tile_log2;
  *buckets = p.nb;
  *emit_path = p.direct ? 0u : (p.split ? 4u : (p.via_bitvec ? 2u : (p.sparse ? 3u : 1u)));
  return BITSORT_OK;
}

}  // extern "C"
