// Bulk query of a PHOBIC MPHF on the device (Sec. 4, "Hash Function": the position of key x with
// pilot p in a partition of m slots is (h(x, floor(p / m)) + p) mod m, plus the partition offset).
//
// One thread per key.  Per key: hash -> partition j -> two offset residues (adjacent, compact) ->
// bucket i by the tabulated bucket function -> encoder i entry j (Compact: one fixed-width field;
// Rice: low bits plus the unary high part located through the select samples) -> position.
// The image (tens of MB at 10^8 keys) stays resident; the accesses per key are a handful of
// dependent cache-line reads that mostly hit the L2 / Infinity Cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <cstring>
#include <string>
#include <vector>
#include <type_traits>

#include "phobic_internal.h"

namespace phobic {
namespace {

constexpr int kQBlock = 256;

// From the select entry e of the block holding one ta: the position of a one at or before one ta
// (the block's sample, or its sub-sample when ta lies past one and the distance was stored), and in
// r how many ones separate the two.
__device__ __forceinline__ uint64_t sel_start(uint64_t e, uint64_t ta, uint32_t& r) {
  const uint32_t left = (uint32_t)(ta % kSelBlock), k = left / kSelSub;
  const uint32_t rel = k ? (uint32_t)(e >> (32 + 10 * (k - 1))) & 1023u : kSelRelNone;
  const bool sub = rel != kSelRelNone;
  r = sub ? left % kSelSub : left;
  return (e & 0xFFFFFFFFULL) + (sub ? rel : 0u);
}

// High part q of value t of the unary stream: q = (position of one t) - (position of one t-1) - 1,
// with one -1 at position -1.  The select entry of one t-1 is read without a preceding branch, so
// its load can issue as soon as t is known.
__device__ __forceinline__ uint64_t unary_high(const uint64_t* __restrict__ un, const uint64_t* __restrict__ sel,
                                               uint64_t t) {
  const uint64_t ta = t ? t - 1 : 0;
  const uint64_t e = sel[ta / kSelBlock];
  uint64_t prev;  // position of one t-1, or UINT64_MAX for t = 0
  uint64_t word;
  uint64_t bits;
  if (t == 0) {
    prev = ~0ULL;
    word = 0;
    bits = un[0];
  } else {
    uint32_t r;
    const uint64_t start = sel_start(e, ta, r);
    word = start >> 6;
    bits = un[word] & (~0ULL << (start & 63));
    for (;;) {
      uint32_t c = __popcll(bits);
      if (r < c) break;
      r -= c;
      bits = un[++word];
    }
    prev = word * 64 + select_in_word(bits, r);
    // continue after prev for the next one
    const uint32_t b = (uint32_t)(prev & 63);
    bits = b == 63 ? 0 : (bits & (~0ULL << (b + 1)));
  }
  while (bits == 0) bits = un[++word];
  const uint64_t cur = word * 64 + (uint32_t)(__ffsll((long long)bits) - 1);
  return cur - prev - 1;
}

// The residues of offsets j and j + 1: adjacent fields of woff <= 32 bits lie in one word or in two
// consecutive ones (the section's trailing pad word keeps idx + 1 inside it); the lookup is bound by
// its memory requests, so the second word is read only when the pair straddles.
__device__ __forceinline__ void offset_pair(const uint64_t* __restrict__ offs, uint64_t j, uint32_t woff,
                                            uint64_t& r0, uint64_t& r1) {
  if (woff == 0) {
    r0 = r1 = 0;
  } else if (woff <= 32) {
    const uint64_t pos = j * woff, idx = pos >> 6;
    const uint32_t sh = (uint32_t)(pos & 63);
    const uint64_t w0 = offs[idx];
    const uint64_t w1 = sh + 2 * woff > 64 ? offs[idx + 1] : 0;  // only a straddling pair reads it
    const uint64_t lo64 = sh ? ((w0 >> sh) | (w1 << (64 - sh))) : w0;  // bits [pos, pos + 64)
    const uint64_t mask = (1ULL << woff) - 1;
    r0 = lo64 & mask;
    r1 = (lo64 >> woff) & mask;
  } else {
    r0 = get_bits(offs, j * woff, woff);
    r1 = get_bits(offs, (j + 1) * woff, woff);
  }
}

__device__ __forceinline__ uint64_t query_code(const QueryArgs& a, uint64_t hi, uint64_t lo) {
  if (a.n == 0) return 0;
  const uint64_t* __restrict__ T = a.table;
  const uint64_t* __restrict__ enc = a.img + a.sec_enc;
  const uint64_t* __restrict__ offs = a.img + a.sec_off;
  // The pilot's fields depend on (i, j) only, not on the offsets: the offset pair, the low bits and
  // the select sample are independent reads that are in flight together.
  const uint64_t j = __umul64hi(hi, a.K);
  const uint32_t i = bucket_of(lo, T, a.B);
  const uint64_t e = enc[i];
  const uint32_t w = (uint32_t)(e & 0xFF);
  uint64_t r0, r1;
  offset_pair(offs, j, a.woff, r0, r1);
  uint64_t p = get_bits(a.img + a.sec_data, (e >> 8) + j * w, w);
  if (a.coding == PHOBIC_IC_RICE && i >= a.ncompact) {  // encoders below ncompact are Compact
    const uint64_t q = unary_high(a.img + a.sec_unary, a.img + a.sec_sel, (uint64_t)(i - a.ncompact) * a.K + j);
    p |= q << w;
  }
  const uint64_t o0 = expected_offset(j, a.R) + (uint64_t)a.dmin + r0;
  const uint64_t o1 = expected_offset(j + 1, a.R) + (uint64_t)a.dmin + r1;
  const uint32_t m = (uint32_t)(o1 - o0);
  if (m == 0) return o0 < a.n ? o0 : a.n - 1;  // only a non-member reaches an empty partition
  // pilots are at most 2^32 - 1, so 32-bit division is exact
  const uint32_t p32 = (uint32_t)p;
  const uint32_t s = p32 / m;
  const uint32_t d = p32 - s * m;
  uint32_t pos = pos_hash(fingerprint(hi, lo), (uint64_t)(s + 1) * kPhi64, m) + d;
  if (pos >= m) pos -= m;
  const uint64_t g = o0 + pos;
  if (g < a.n) return g;
  return get_bits(a.img + a.sec_remap, (g - a.n) * a.wremap, a.wremap);
}

// bucket_of over a table held in 64-bit words, or in 32-bit words where the last point, 2^32, reads
// as 0: the difference of two points is then still right modulo 2^32, and it is below 2^32.  Every
// other point is below 2^32 (the bucket functions stay below 1 short of x = 1 by far more than 2^-32).
__device__ __forceinline__ uint32_t bucket_of_tab(uint64_t lo, const uint64_t* __restrict__ T, uint32_t B) {
  return bucket_of(lo, T, B);
}
__device__ __forceinline__ uint32_t bucket_of_tab(uint64_t lo, const uint32_t* __restrict__ T, uint32_t B) {
  const uint32_t k = (uint32_t)(lo >> 53);
  const uint64_t f = (lo >> 21) & 0xFFFFFFFFULL;
  const uint32_t t0 = T[k], t1 = T[k + 1];
  const uint64_t y = (uint64_t)t0 + (((uint64_t)(uint32_t)(t1 - t0) * f) >> 32);
  const uint32_t b = (uint32_t)((y * B) >> 32);
  return b < B - 1 ? b : B - 1;
}

// kN lookups per thread in lockstep: every stage issues the reads of all kN lookups before any of
// them is consumed, so one wavefront keeps kN times as many independent cache-line reads in flight
// (the query is bound by the latency of its chain of dependent reads, not by bandwidth).  Same
// arithmetic as query_code.
template <int kN, typename TabT>
__device__ __forceinline__ void query_codes(const QueryArgs& a, const TabT* __restrict__ T,
                                            const uint64_t* __restrict__ E, const uint64_t (&hi)[kN],
                                            const uint64_t (&lo)[kN], uint64_t (&res)[kN]) {
  const uint64_t* __restrict__ offs = a.img + a.sec_off;
  const uint64_t* __restrict__ un = a.img + a.sec_unary;
  const uint64_t* __restrict__ sel = a.img + a.sec_sel;
  const bool rice = a.coding == PHOBIC_IC_RICE;
  uint64_t j[kN], e[kN], p[kN], r0[kN], r1[kN];
  uint32_t i[kN];
#pragma unroll
  for (int q = 0; q < kN; q++) {
    j[q] = __umul64hi(hi[q], a.K);
    i[q] = bucket_of_tab(lo[q], T, a.B);
  }
#pragma unroll
  for (int q = 0; q < kN; q++) e[q] = E[i[q]];
  // offsets, low bits and select samples: independent of each other.  A lookup whose encoder is
  // Rice (u) reads the unary stream at its value t = (i - ncompact) K + j; one of a Compact encoder
  // (all of a Compact image, the first ncompact of a mixed one) is done with its field.
  uint64_t t[kN], ta[kN], sample[kN];
  bool u[kN];
#pragma unroll
  for (int q = 0; q < kN; q++) {
    offset_pair(offs, j[q], a.woff, r0[q], r1[q]);
    const uint32_t w = (uint32_t)(e[q] & 0xFF);
    p[q] = get_bits(a.img + a.sec_data, (e[q] >> 8) + j[q] * w, w);
    u[q] = rice && i[q] >= a.ncompact;
    t[q] = u[q] ? (uint64_t)(i[q] - a.ncompact) * a.K + j[q] : 0;
    ta[q] = t[q] ? t[q] - 1 : 0;
    sample[q] = u[q] ? sel[ta[q] / kSelBlock] : 0;
  }
  if (rice) {
    uint64_t word[kN], bits[kN], prev[kN];
    uint32_t r[kN];
    bool found[kN];
#pragma unroll
    for (int q = 0; q < kN; q++) {
      const uint64_t start = sel_start(sample[q], ta[q], r[q]);
      word[q] = t[q] ? start >> 6 : 0;
      bits[q] = u[q] ? un[word[q]] : 1;  // a Compact lookup keeps a set bit: no reads below
      if (t[q]) bits[q] &= ~0ULL << (start & 63);
      found[q] = t[q] == 0;
    }
    // the one of value t - 1: skip r ones from the sample
    for (bool more = true; more;) {
      more = false;
#pragma unroll
      for (int q = 0; q < kN; q++) {
        if (!found[q]) {
          const uint32_t c = __popcll(bits[q]);
          if (r[q] < c) {
            found[q] = true;
          } else {
            r[q] -= c;
            bits[q] = un[++word[q]];
            more = true;
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kN; q++) {
      if (t[q] == 0) {
        prev[q] = ~0ULL;
      } else {
        prev[q] = word[q] * 64 + select_in_word(bits[q], r[q]);
        const uint32_t b = (uint32_t)(prev[q] & 63);
        bits[q] = b == 63 ? 0 : (bits[q] & (~0ULL << (b + 1)));
      }
    }
    // the one of value t: the next set bit
    for (bool more = true; more;) {
      more = false;
#pragma unroll
      for (int q = 0; q < kN; q++) {
        if (bits[q] == 0) {
          bits[q] = un[++word[q]];
          more = true;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kN; q++) {
      const uint64_t cur = word[q] * 64 + (uint32_t)(__ffsll((long long)bits[q]) - 1);
      if (u[q]) p[q] |= (cur - prev[q] - 1) << (uint32_t)(e[q] & 0xFF);
    }
  }
#pragma unroll
  for (int q = 0; q < kN; q++) {
    const uint64_t o0 = expected_offset(j[q], a.R) + (uint64_t)a.dmin + r0[q];
    const uint64_t o1 = expected_offset(j[q] + 1, a.R) + (uint64_t)a.dmin + r1[q];
    const uint32_t m = (uint32_t)(o1 - o0);
    if (m == 0) {  // only a non-member reaches an empty partition
      res[q] = o0 < a.n ? o0 : a.n - 1;
      continue;
    }
    const uint32_t p32 = (uint32_t)p[q];
    const uint32_t s = p32 / m;
    const uint32_t d = p32 - s * m;
    uint32_t pos = pos_hash(fingerprint(hi[q], lo[q]), (uint64_t)(s + 1) * kPhi64, m) + d;
    if (pos >= m) pos -= m;
    const uint64_t g = o0 + pos;
    res[q] = g < a.n ? g : get_bits(a.img + a.sec_remap, (g - a.n) * a.wremap, a.wremap);
  }
}

constexpr int kQN = 4;
constexpr uint32_t kQEncLds = 1024;  // encoders the LDS-staged query holds

// Thread x handles keys x, x + stride, ..., kQN of them per round.  kLds: the bucket-function table
// (as 32-bit words) and the encoder words (B <= kQEncLds) are read from LDS, where the workgroup
// copies them first: a wavefront's read of either touches dozens of cache lines, and the lookup is
// bound by its cache requests (10.9 KB per workgroup at B = 358, 7% off the query time at 10^8 keys).
template <bool kLds, typename TabT = typename std::conditional<kLds, uint32_t, uint64_t>::type>
__global__ __launch_bounds__(kQBlock) void k_query_u64(QueryArgs a, const uint64_t* __restrict__ keys, uint64_t n,
                                                        uint64_t* __restrict__ out) {
  if (a.n == 0) {
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n; x += (uint64_t)gridDim.x * blockDim.x)
      out[x] = 0;
    return;
  }
  __shared__ TabT sT[kLds ? kTableIntervals + 1 : 1];
  __shared__ uint64_t sE[kLds ? kQEncLds : 1];
  const uint64_t* E = a.img + a.sec_enc;
  if (kLds) {
    for (uint32_t x = threadIdx.x; x <= kTableIntervals; x += kQBlock) sT[x] = (TabT)a.table[x];
    for (uint32_t x = threadIdx.x; x < a.B; x += kQBlock) sE[x] = E[x];
    __syncthreads();
    E = sE;
  }
  const TabT* T = kLds ? (const TabT*)sT : (const TabT*)a.table;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t x0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x0 < n; x0 += stride * kQN) {
    uint64_t hi[kQN], lo[kQN], res[kQN];
#pragma unroll
    for (int q = 0; q < kQN; q++) {
      const uint64_t x = x0 + q * stride;
      hash_key_u64(keys[x < n ? x : x0], a.seed, hi[q], lo[q]);
    }
    query_codes<kQN, TabT>(a, T, E, hi, lo, res);
#pragma unroll
    for (int q = 0; q < kQN; q++) {
      const uint64_t x = x0 + q * stride;
      if (x < n) out[x] = res[q];
    }
  }
}

__global__ __launch_bounds__(kQBlock) void k_query_str(QueryArgs a, const uint8_t* __restrict__ bytes,
                                                       const uint64_t* __restrict__ offs, uint64_t n,
                                                       uint64_t* __restrict__ out) {
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n; x += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t s0 = offs[x], s1 = offs[x + 1];
    uint64_t hi, lo;
    hash_key_str(bytes + s0, s1 - s0, a.seed, hi, lo);
    out[x] = query_code(a, hi, lo);
  }
}

// Several requests in one launch: blocks [bstart[r], bstart[r+1]) serve request r.
struct QueryJob {
  QueryArgs qa;
  const uint64_t* keys;
  uint64_t* out;
  uint64_t n;
};
constexpr uint32_t kMultiItems = 4;

// Lookups first + t kQBlock + threadIdx.x (t < kMultiItems) of request jb, in lockstep (query_codes).
// The block exists for the request, so its first lookup is in range and stands in for those past the
// end.
template <typename TabT>
__device__ __forceinline__ void multi_items(const QueryJob& jb, const TabT* T, const uint64_t* E, uint64_t first) {
  uint64_t hi[kMultiItems], lo[kMultiItems], res[kMultiItems];
#pragma unroll
  for (uint32_t t = 0; t < kMultiItems; t++) {
    const uint64_t x = first + t * kQBlock + threadIdx.x;
    hash_key_u64(jb.keys[x < jb.n ? x : first], jb.qa.seed, hi[t], lo[t]);
  }
  query_codes<(int)kMultiItems, TabT>(jb.qa, T, E, hi, lo, res);
#pragma unroll
  for (uint32_t t = 0; t < kMultiItems; t++) {
    const uint64_t x = first + t * kQBlock + threadIdx.x;
    if (x < jb.n) jb.out[x] = res[t];
  }
}

// As k_query_u64 (the bucket table and encoder words staged in LDS when B <= kQEncLds), one request
// per block.
__global__ __launch_bounds__(kQBlock) void k_query_multi(const QueryJob* __restrict__ jobs,
                                                         const uint64_t* __restrict__ bstart, uint32_t count) {
  __shared__ uint32_t sj;
  __shared__ uint32_t sT[kTableIntervals + 1];
  __shared__ uint64_t sE[kQEncLds];
  if (threadIdx.x == 0) {
    uint32_t lo = 0, hi = count;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (bstart[mid] <= blockIdx.x) lo = mid; else hi = mid;
    }
    sj = lo;
  }
  __syncthreads();
  const QueryJob& jb = jobs[sj];
  const uint64_t first = (uint64_t)(blockIdx.x - bstart[sj]) * kQBlock * kMultiItems;
  if (jb.qa.n == 0) {  // an empty MPHF: every key maps to 0
    for (uint32_t t = 0; t < kMultiItems; t++) {
      const uint64_t x = first + t * kQBlock + threadIdx.x;
      if (x < jb.n) jb.out[x] = 0;
    }
    return;
  }
  const uint64_t* E = jb.qa.img + jb.qa.sec_enc;
  if (jb.qa.B <= kQEncLds) {
    for (uint32_t x = threadIdx.x; x <= kTableIntervals; x += kQBlock) sT[x] = (uint32_t)jb.qa.table[x];
    for (uint32_t x = threadIdx.x; x < jb.qa.B; x += kQBlock) sE[x] = E[x];
    __syncthreads();
    multi_items<uint32_t>(jb, sT, sE, first);
  } else {
    multi_items<uint64_t>(jb, jb.qa.table, E, first);
  }
}

// ---------------------------------------------------------------------------------------------
// Allocation-free multi-request query: the job table lives in `scratch`, a fixed device array of
// this library (one per GPU, kept until the process ends), instead of a pool allocation.  Its
// layout: kNoAllocRequests jobs, then kNoAllocRequests block starts.
// ---------------------------------------------------------------------------------------------
constexpr uint32_t kNoAllocRequests = 4096;
constexpr size_t kNoAllocJobBytes = (size_t)kNoAllocRequests * sizeof(QueryJob);
constexpr size_t kNoAllocBytes = kNoAllocJobBytes + (size_t)kNoAllocRequests * sizeof(uint64_t);
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;                   // guards the table below and the host staging
void* g_noalloc_dev[kNoAllocDevices] = {};  // device address of `scratch` per device
// Host staging of one call's table (pageable; a copy from it is staged before the copy call returns).
alignas(64) uint8_t g_noalloc_host[kNoAllocBytes];

uint32_t query_grid(uint64_t n, uint32_t per_thread = 1) {
  uint64_t g = (n + (uint64_t)kQBlock * per_thread - 1) / ((uint64_t)kQBlock * per_thread);
  return (uint32_t)(g < 1 ? 1 : (g > 1048576 ? 1048576 : g));
}

}  // namespace
}  // namespace phobic

using namespace phobic;

extern "C" phobic_status phobic_query_u64(const phobic_mphf* h, const uint64_t* d_keys, uint64_t n, uint64_t* d_pos,
                                          void* hip_stream) {
  if (!h) return fail(PHOBIC_E_INVALID, "null handle");
  if (n == 0) return PHOBIC_OK;
  if (!d_keys || !d_pos) return fail(PHOBIC_E_INVALID, "null key or output pointer");
  if (h->qa.B <= kQEncLds)
    hipLaunchKernelGGL((k_query_u64<true>), dim3(query_grid(n, kQN)), dim3(kQBlock), 0, (hipStream_t)hip_stream,
                       h->qa, d_keys, n, d_pos);
  else
    hipLaunchKernelGGL((k_query_u64<false>), dim3(query_grid(n, kQN)), dim3(kQBlock), 0, (hipStream_t)hip_stream,
                       h->qa, d_keys, n, d_pos);
  PHOBIC_HIP(hipGetLastError());
  return PHOBIC_OK;
}

extern "C" phobic_status phobic_query_str(const phobic_mphf* h, const uint8_t* d_bytes, const uint64_t* d_offsets,
                                          uint64_t n, uint64_t* d_pos, void* hip_stream) {
  if (!h) return fail(PHOBIC_E_INVALID, "null handle");
  if (n == 0) return PHOBIC_OK;
  if (!d_bytes || !d_offsets || !d_pos) return fail(PHOBIC_E_INVALID, "null key or output pointer");
  hipLaunchKernelGGL(k_query_str, dim3(query_grid(n)), dim3(kQBlock), 0, (hipStream_t)hip_stream, h->qa, d_bytes,
                     d_offsets, n, d_pos);
  PHOBIC_HIP(hipGetLastError());
  return PHOBIC_OK;
}

extern "C" phobic_status phobic_query_multi_u64(const phobic_mphf* const* h_handles, const uint64_t* const* h_keys,
                                                const uint64_t* h_counts, uint64_t* const* h_outs, uint32_t count,
                                                void* hip_stream) {
  if (count == 0) return PHOBIC_OK;
  if (!h_handles || !h_keys || !h_counts || !h_outs) return fail(PHOBIC_E_INVALID, "null argument");
  std::vector<QueryJob> jobs;
  std::vector<uint64_t> bstart;
  uint64_t blocks = 0;
  for (uint32_t r = 0; r < count; r++) {
    if (!h_handles[r]) return fail(PHOBIC_E_INVALID, "null handle in request " + std::to_string(r));
    const uint64_t n = h_counts[r];
    if (n == 0) continue;
    if (!h_keys[r] || !h_outs[r]) return fail(PHOBIC_E_INVALID, "null pointer in request " + std::to_string(r));
    jobs.push_back(QueryJob{h_handles[r]->qa, h_keys[r], h_outs[r], n});
    bstart.push_back(blocks);
    blocks += (n + (uint64_t)kQBlock * kMultiItems - 1) / ((uint64_t)kQBlock * kMultiItems);
  }
  if (jobs.empty()) return PHOBIC_OK;
  if (blocks > 0x7FFFFFFFULL) return fail(PHOBIC_E_INVALID, "too many keys in one call");
  hipStream_t st = (hipStream_t)hip_stream;
  const size_t jbytes = jobs.size() * sizeof(QueryJob), bbytes = bstart.size() * sizeof(uint64_t);
  // per-thread pinned staging; the event of its last copy guards reuse
  struct Staging {
    void* p = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
  };
  thread_local Staging stg;
  if (!stg.ev) PHOBIC_HIP(hipEventCreateWithFlags(&stg.ev, hipEventDisableTiming));
  PHOBIC_HIP(hipEventSynchronize(stg.ev));
  if (stg.cap < jbytes + bbytes) {
    if (stg.p) (void)hipHostFree(stg.p);
    stg.p = nullptr;
    stg.cap = 0;
    const size_t cap = std::max<size_t>(jbytes + bbytes, 1 << 16);
    PHOBIC_HIP(hipHostMalloc(&stg.p, cap, hipHostMallocDefault));
    stg.cap = cap;
  }
  std::memcpy(stg.p, jobs.data(), jbytes);
  std::memcpy((char*)stg.p + jbytes, bstart.data(), bbytes);
  void* dbuf = nullptr;
  PHOBIC_HIP(pool_alloc(&dbuf, jbytes + bbytes, st));
  hipError_t e = hipMemcpyAsync(dbuf, stg.p, jbytes + bbytes, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipEventRecord(stg.ev, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_query_multi, dim3((uint32_t)blocks), dim3(kQBlock), 0, st, (const QueryJob*)dbuf,
                       (const uint64_t*)((char*)dbuf + jbytes), (uint32_t)jobs.size());
    e = hipGetLastError();
  }
  (void)hipFreeAsync(dbuf, st);
  if (e != hipSuccess) return fail(PHOBIC_E_DEVICE, std::string("query_multi: ") + hipGetErrorString(e));
  return PHOBIC_OK;
}

extern "C" phobic_status phobic_query_multi_u64_noalloc(const phobic_mphf* const* h_handles,
                                                        const uint64_t* const* h_keys, const uint64_t* h_counts,
                                                        uint64_t* const* h_outs, uint32_t count, void* hip_stream) {
  if (count == 0) return PHOBIC_OK;
  if (!h_handles || !h_keys || !h_counts || !h_outs) return fail(PHOBIC_E_INVALID, "null argument");
  if (count > kNoAllocRequests)
    return fail(PHOBIC_E_INVALID, "at most " + std::to_string(kNoAllocRequests) + " requests per call");
  int dev = 0;
  PHOBIC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocDevices) return fail(PHOBIC_E_INVALID, "device index out of range");
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_dev[dev]) {  // once per device, with that device current: the array's own address
    void* ptr = nullptr;
    PHOBIC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(PHOBIC_E_DEVICE, "no device address for the query scratch array");
    g_noalloc_dev[dev] = ptr;
  }
  uint8_t* dscr = (uint8_t*)g_noalloc_dev[dev];
  QueryJob* jobs = (QueryJob*)g_noalloc_host;
  uint64_t* bstart = (uint64_t*)(g_noalloc_host + kNoAllocJobBytes);
  uint32_t nj = 0;
  uint64_t blocks = 0;
  for (uint32_t r = 0; r < count; r++) {
    if (!h_handles[r]) return fail(PHOBIC_E_INVALID, "null handle in request " + std::to_string(r));
    const uint64_t n = h_counts[r];
    if (n == 0) continue;
    if (!h_keys[r] || !h_outs[r]) return fail(PHOBIC_E_INVALID, "null pointer in request " + std::to_string(r));
    jobs[nj] = QueryJob{h_handles[r]->qa, h_keys[r], h_outs[r], n};
    bstart[nj] = blocks;
    nj++;
    blocks += (n + (uint64_t)kQBlock * kMultiItems - 1) / ((uint64_t)kQBlock * kMultiItems);
  }
  if (nj == 0) return PHOBIC_OK;
  if (blocks > 0x7FFFFFFFULL) return fail(PHOBIC_E_INVALID, "too many keys in one call");
  hipStream_t st = (hipStream_t)hip_stream;
  PHOBIC_HIP(hipMemcpyAsync(dscr, jobs, nj * sizeof(QueryJob), hipMemcpyHostToDevice, st));
  PHOBIC_HIP(hipMemcpyAsync(dscr + kNoAllocJobBytes, bstart, nj * sizeof(uint64_t), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_query_multi, dim3((uint32_t)blocks), dim3(kQBlock), 0, st, (const QueryJob*)dscr,
                     (const uint64_t*)(dscr + kNoAllocJobBytes), nj);
  PHOBIC_HIP(hipGetLastError());
  return PHOBIC_OK;
}
