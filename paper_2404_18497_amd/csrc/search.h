// Pilot search (Sec. 4, Sec. 4.2; Alg. 1): the interface between the build orchestration and the
// search kernels.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "phobic.h"

namespace phobic {

struct SearchArgs {
  const uint64_t* fp;     // fingerprints in processing order, partition-contiguous
  const uint64_t* off;    // key offsets, K + 1
  const uint64_t* toff;   // table offsets, K + 1
  const uint32_t* blist;  // per partition: (size << 16 | bucket) in processing order
  const uint32_t* nbk;    // non-empty buckets per partition
  uint32_t* pilots;       // one MPHF: partition-major, pilots[j * B + i]; several: see owner
  uint32_t* err;          // bit (1 << status) for every error met
  uint64_t* taken;        // occupancy bitmap of all tables (alpha < 1), else null
  uint64_t K;
  uint64_t limit;
  uint32_t B;
  uint32_t f2_words;      // 32-bit words of F2 (multiple of 4)
  uint32_t scr_words;     // 32-bit words of the collision scratch (multiple of 4)
  uint32_t rb_cap;        // 32-bit position entries (multiple of 4, at least kSearchMinPositions)
  uint32_t bl_cap;        // 32-bit entries of the pilot row (multiple of 4); 0 on the wide path
  uint32_t cm_cap;        // 64-bit collision masks
  uint32_t max_m;         // the largest table (slots) the LDS layout holds
  uint32_t max_bucket;    // the largest bucket (keys) the LDS layout holds
  uint32_t wide;          // 1: pilot row in global memory and F2 unshifted (wide partitions, one MPHF)
  uint32_t wave_lds;      // bytes of LDS per wavefront (multiple of 16), see size_search_lds
  // several MPHFs at once: partition J belongs to MPHF owner[J], whose partitions start at
  // Kbase[t] (K_t of them) and whose pilots start at B * Kbase[t]; null for a single MPHF
  const uint32_t* owner;
  const uint64_t* Kbase;
  const uint64_t* Kt;
  // persistent launch: partitions are taken grab at a time from *queue; null = one per wavefront
  unsigned long long* queue;
  uint32_t grab;
  unsigned long long* fail_part;  // non-null: receives the lowest failing partition index (atomic min)
  const uint32_t* order;          // non-null: the launch takes partitions in this order (one MPHF)
};

// Launches the search over `items` partitions (sa.K of them in the partition index space) on the
// stream with the configured launch shape; `queue` is one device word used by the persistent shape.
hipError_t launch_search(SearchArgs& sa, uint64_t items, hipStream_t st, unsigned long long* queue);

// Orders the K partitions of one MPHF by an estimate of their search cost, largest first, into
// order[0 .. K) (scratch: order_scratch_words(K) words); sets sa.order.  The order changes no result.
hipError_t order_partitions(SearchArgs& sa, uint32_t* order, uint32_t* scratch, hipStream_t st);
inline uint64_t order_scratch_words(uint64_t K) { return 512 + (K + 3) / 4; }  // histogram, cursors, a byte per partition

// The position buffer holds at least one entry per lane (a small bucket's seeds are hashed 64
// positions at a time), and each wavefront keeps kSearchCtxBytes of argument fields in LDS.
constexpr uint32_t kSearchMinPositions = 64;
constexpr uint32_t kSearchCtxBytes = 64;

// Sizes the per-wavefront LDS layout for tables of up to mm slots and buckets of up to mb keys
// (mm, mb >= 1): F2 (outside the wide path also its copy shifted by one word), collision scratch,
// positions, pilot row, collision masks, argument context.  Sets the size fields, max_m,
// max_bucket and wide.
inline void size_search_lds(SearchArgs& sa, uint32_t mm, uint32_t mb, uint32_t B, bool wide) {
  auto up4 = [](uint32_t v) { return (v + 3) & ~3u; };
  sa.f2_words = up4((2 * mm + 127) / 32 + 1);
  sa.scr_words = up4((mm + 31) / 32 + 1);
  sa.rb_cap = up4(mb) + 4 > kSearchMinPositions ? up4(mb) + 4 : kSearchMinPositions;
  sa.bl_cap = wide ? 0u : up4(B);  // wide: pilots in global memory
  sa.cm_cap = (mb + 63) / 64 + 1;
  sa.max_m = mm;
  sa.max_bucket = mb;
  sa.wide = wide ? 1u : 0u;
  const uint32_t f2_copies = wide ? 1u : 2u;
  sa.wave_lds = ((sa.f2_words * f2_copies + sa.scr_words + sa.rb_cap + sa.bl_cap) * 4 + sa.cm_cap * 8 +
                 kSearchCtxBytes + 15) & ~15u;
}

// Error bit of a partition or bucket larger than the search's LDS layout was sized for (the build
// then repeats with exact sizes); beyond the phobic_status values.
constexpr uint32_t kErrResize = 16;

}  // namespace phobic
