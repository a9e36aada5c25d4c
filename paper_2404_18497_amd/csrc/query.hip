// Bulk query of a PHOBIC MPHF on the device (Sec. 4, "Hash Function": the position of key x with
// pilot p in a partition of m slots is (h(x, floor(p / m)) + p) mod m, plus the partition offset).
//
// One thread per key.  Per key: hash -> partition j -> two offset residues (adjacent, compact) ->
// bucket i by the tabulated bucket function -> encoder i entry j (Compact: one fixed-width field;
// Rice: low bits plus the unary high part located through the select samples) -> position.
// The image (tens of MB at 10^8 keys) stays resident; the accesses per key are a handful of
// dependent cache-line reads that mostly hit the L2 / Infinity Cache.
#include <hip/hip_runtime.h>

#include "phobic_internal.h"

namespace phobic {
namespace {

constexpr int kQBlock = 256;

// Position of the r-th set bit (r from 0) of a 64-bit word that has more than r set bits.
__device__ __forceinline__ uint32_t select_in_word(uint64_t x, uint32_t r) {
  uint32_t pos = 0;
  uint32_t c = __popc((uint32_t)x);
  if (r >= c) { r -= c; x >>= 32; pos += 32; }
  c = __popc((uint32_t)x & 0xFFFFu);
  if (r >= c) { r -= c; x >>= 16; pos += 16; }
  c = __popc((uint32_t)x & 0xFFu);
  if (r >= c) { r -= c; x >>= 8; pos += 8; }
  c = __popc((uint32_t)x & 0xFu);
  if (r >= c) { r -= c; x >>= 4; pos += 4; }
  c = __popc((uint32_t)x & 0x3u);
  if (r >= c) { r -= c; x >>= 2; pos += 2; }
  c = (uint32_t)(x & 1u);
  if (r >= c) { pos += 1; }
  return pos;
}

// High part q of value t of the unary stream: q = (position of one t) - (position of one t-1) - 1,
// with one -1 at position -1.  Starts from the sample of one number 256 floor((t-1)/256).
__device__ __forceinline__ uint64_t unary_high(const uint64_t* __restrict__ un, const uint32_t* __restrict__ sel,
                                               uint64_t t) {
  uint64_t prev;  // position of one t-1, or UINT64_MAX for t = 0
  uint64_t word;
  uint64_t bits;
  if (t == 0) {
    prev = ~0ULL;
    word = 0;
    bits = un[0];
  } else {
    const uint64_t ta = t - 1;
    const uint64_t s = ta / kSelEvery;
    uint64_t pos = sel[s];
    uint32_t r = (uint32_t)(ta - s * kSelEvery);
    word = pos >> 6;
    bits = un[word] & (~0ULL << (pos & 63));
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

__device__ __forceinline__ uint64_t query_code(const QueryArgs& a, uint64_t hi, uint64_t lo) {
  if (a.n == 0) return 0;
  const uint64_t j = __umul64hi(hi, a.K);
  const uint64_t* offs = a.img + a.sec_off;
  const uint64_t o0 = expected_offset(j, a.R) + (uint64_t)a.dmin + get_bits(offs, j * a.woff, a.woff);
  const uint64_t o1 = expected_offset(j + 1, a.R) + (uint64_t)a.dmin + get_bits(offs, (j + 1) * a.woff, a.woff);
  const uint32_t m = (uint32_t)(o1 - o0);
  if (m == 0) return o0 < a.n ? o0 : a.n - 1;  // only a non-member reaches an empty partition
  const uint32_t i = bucket_of(lo, a.table, a.B);
  const uint64_t e = a.img[a.sec_enc + i];
  const uint32_t w = (uint32_t)(e & 0xFF);
  uint64_t p = get_bits(a.img + a.sec_data, (e >> 8) + j * w, w);
  if (a.coding == PHOBIC_IC_RICE) {
    const uint64_t q = unary_high(a.img + a.sec_unary, (const uint32_t*)(a.img + a.sec_sel), (uint64_t)i * a.K + j);
    p |= q << w;
  }
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

__global__ __launch_bounds__(kQBlock) void k_query_u64(QueryArgs a, const uint64_t* __restrict__ keys, uint64_t n,
                                                       uint64_t* __restrict__ out) {
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n; x += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t hi, lo;
    hash_key_u64(keys[x], a.seed, hi, lo);
    out[x] = query_code(a, hi, lo);
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

uint32_t query_grid(uint64_t n) {
  uint64_t g = (n + kQBlock - 1) / kQBlock;
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
  hipLaunchKernelGGL(k_query_u64, dim3(query_grid(n)), dim3(kQBlock), 0, (hipStream_t)hip_stream, h->qa, d_keys, n,
                     d_pos);
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
