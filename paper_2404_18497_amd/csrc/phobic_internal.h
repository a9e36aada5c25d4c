// Internal declarations of the MI355X PHOBIC library: image layout, handle, error plumbing and the
// device helpers shared by the build and query kernels.  Everything here follows the specification
// of the key hash, the bucket function and the image; none of it is shared with the CPU oracle.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <string>
#include <vector>

#include "phobic.h"

namespace phobic {

// ---------------------------------------------------------------------------------------------
// Limits of the device path.  One partition is handled by one workgroup whose working set lives in
// LDS: the per-key bucket records of the bucket sort (4 bytes per key) and the free-slot bitmap of
// the search.  Larger partitions or more buckets are reported as PHOBIC_E_CAPACITY.
// ---------------------------------------------------------------------------------------------
constexpr uint32_t kMaxPartitionKeys = 8192;  // n_j
constexpr uint32_t kMaxTableSlots = 16384;    // m_j (alpha < 1 enlarges n_j)
constexpr uint32_t kMaxBuckets = 2048;        // B
// Wide partitions (beyond the three limits above) take a path that keeps only the slot bitmaps and
// the current bucket's positions in LDS, one workgroup per partition; the LDS of one workgroup then
// bounds m_j (and the bucket sort's B), and the position encoding of the search m_j < 2^19.
constexpr uint32_t kWideMaxBuckets = 65535;
constexpr uint64_t kWideMaxTableSlots = 1ULL << 19;
constexpr uint32_t kTableIntervals = 2048;    // bucket-function table: 2048 intervals, 2049 points
// Select samples of the unary stream, one 64-bit entry per kSelBlock ones: entry s holds the position
// of one number kSelBlock s in its low 32 bits and, for k = 1, 2, 3, the distance from there to one
// number kSelBlock s + kSelSub k in the 10-bit field at bit 32 + 10 (k - 1); kSelRelNone when the
// distance does not fit, 0 for ones past the end of the stream.
constexpr uint32_t kSelBlock = 256;
constexpr uint32_t kSelSub = 64;
constexpr uint32_t kSelRelNone = 1023;

// Image header word indices (little-endian 64-bit words).
enum : uint32_t {
  kHMagic = 0, kHN, kHK, kHB, kHP, kHLambda, kHAlpha, kHCoding, kHSeed, kHTotal, kHDmin, kHWoff,
  kHSecOff, kHSecEnc, kHSecData, kHSecUnary, kHSecSel, kHSecRemap, kHWremap, kHNremap, kHUbits,
  kHWords, kHR, kHNcompact, kHeaderWords
};
constexpr uint64_t kMagic = 0x33304349424F4850ULL;  // "PHOBIC03"

// Everything a query kernel needs, passed by value.
struct QueryArgs {
  const uint64_t* img;    // device image
  const uint64_t* table;  // device bucket-function table (kTableIntervals + 1 entries)
  uint64_t n, K, R, total;
  int64_t dmin;
  uint64_t sec_off, sec_enc, sec_data, sec_unary, sec_sel, sec_remap;
  uint64_t seed;
  uint32_t B, woff, coding, wremap;
  uint32_t ncompact;  // Rice images: encoders below it are Compact (mixed interleaved coding)
};

}  // namespace phobic

struct phobic_mphf {
  int device = 0;
  uint64_t n = 0, K = 0;
  uint32_t B = 0;
  phobic_params prm{};
  uint64_t* d_image = nullptr;
  uint64_t nwords = 0;
  std::vector<uint64_t> header;   // host copy of the header words
  uint64_t* d_table = nullptr;   // borrowed from the per-device table cache
  uint32_t* d_pilots = nullptr;   // partition-major (j * B + i), only with PHOBIC_FLAG_KEEP_PILOTS
  phobic_build_info info{};
  phobic::QueryArgs qa{};
  std::shared_ptr<void> shared;   // set when d_image lives inside one allocation shared by a batch
};

namespace phobic {

// ---------------------------------------------------------------------------------------------
// Error plumbing (host).
// ---------------------------------------------------------------------------------------------
void set_error(const std::string& msg);
phobic_status fail(phobic_status s, const std::string& msg);
#define PHOBIC_HIP(call)                                                                            \
  do {                                                                                              \
    hipError_t e_ = (call);                                                                         \
    if (e_ != hipSuccess)                                                                           \
      return ::phobic::fail(e_ == hipErrorOutOfMemory ? PHOBIC_E_OOM : PHOBIC_E_DEVICE,              \
                            std::string(#call) + ": " + hipGetErrorString(e_));                    \
  } while (0)

// Header words of an image from its sizes: the section layout follows from them (the same on the
// host and in device planning kernels).  coding_word = coding | bucket function << 8; c = leading
// Compact encoders of a mixed Rice image.
__host__ __device__ inline void fill_header(uint64_t* hdr, uint64_t n, uint64_t K, uint32_t B, uint32_t P,
                                            uint64_t lambda_bits, uint64_t alpha_word, uint64_t coding_word,
                                            uint64_t seed, uint64_t total, int64_t dmin, uint32_t woff,
                                            uint64_t data_bits, uint64_t unary_bits, uint64_t R, uint32_t c) {
  const bool rice = (coding_word & 0xFF) == PHOBIC_IC_RICE;
  const uint64_t nremap = total - n;
  uint32_t wremap = 0;
  for (uint64_t v = n > 1 ? n - 1 : 0; v; v >>= 1) wremap++;  // bit length of n - 1
  const uint64_t nsel = rice ? (K * (B - c) + kSelBlock - 1) / kSelBlock : 0;
  for (uint32_t x = 0; x < kHeaderWords; x++) hdr[x] = 0;
  hdr[kHMagic] = kMagic;
  hdr[kHN] = n;
  hdr[kHK] = K;
  hdr[kHB] = B;
  hdr[kHP] = P;
  hdr[kHLambda] = lambda_bits;
  hdr[kHAlpha] = alpha_word;
  hdr[kHCoding] = coding_word;
  hdr[kHSeed] = seed;
  hdr[kHTotal] = total;
  hdr[kHDmin] = (uint64_t)dmin;
  hdr[kHWoff] = woff;
  hdr[kHSecOff] = kHeaderWords;
  hdr[kHSecEnc] = hdr[kHSecOff] + ((K + 1) * woff + 63) / 64 + 1;
  hdr[kHSecData] = hdr[kHSecEnc] + B + 1;
  hdr[kHSecUnary] = hdr[kHSecData] + (data_bits + 63) / 64 + 1;
  hdr[kHSecSel] = hdr[kHSecUnary] + (rice ? (unary_bits + 63) / 64 + 1 : 0);
  hdr[kHSecRemap] = hdr[kHSecSel] + (rice ? nsel + 1 : 0);
  hdr[kHWremap] = wremap;
  hdr[kHNremap] = nremap;
  hdr[kHUbits] = rice ? unary_bits : 0;
  hdr[kHWords] = hdr[kHSecRemap] + (nremap ? (nremap * wremap + 63) / 64 + 1 : 0);
  hdr[kHR] = R;
  hdr[kHNcompact] = rice ? c : 0;
}

// Kiely's Golomb-Rice parameter depends on the mean mu = sum / count only and does not decrease with
// it, so it is fixed by 32 thresholds on mu: b = #{t : mu >= mu_t}.  The thresholds are found once
// on the host from the same double formula (and checked at both sides of each), so a device that
// divides in IEEE double picks exactly the parameter the host would.
struct RiceThresholds {
  double mu[32];
};
const RiceThresholds& rice_thresholds();
__host__ __device__ inline uint32_t rice_from_thresholds(uint64_t sum, uint64_t count, const RiceThresholds& t) {
  if (sum == 0 || count == 0) return 0;
  const double mu = (double)sum / (double)count;
  uint32_t b = 0;
  while (b < 32 && mu >= t.mu[b]) b++;
  return b;
}

// Host planning shared by build and deserialize.
phobic_status validate_params(const phobic_params* p, uint32_t* B);
uint64_t num_partitions(uint64_t n, uint32_t P);
void bucket_table(double lambda, uint32_t P, uint32_t an, uint32_t ad, uint32_t fn, uint64_t* T);
uint32_t rice_parameter(uint64_t sum, uint64_t count);
phobic_status upload_table(phobic_mphf* h, hipStream_t st);
std::vector<uint64_t> make_header(uint64_t n, uint64_t K, uint32_t B, const phobic_params& prm, uint64_t total,
                                  int64_t dmin, uint32_t woff, uint64_t data_bits, uint64_t unary_bits, uint64_t R);
void fill_query_args(phobic_mphf* h);

// Stream-ordered device memory for images (and short-lived launch buffers) from a per-device pool of
// this library, which keeps up to kPoolKeepBytes of freed memory mapped for the next allocation:
// repeated builds then reuse pages instead of mapping fresh ones.  Released with hipFreeAsync.
constexpr uint64_t kPoolKeepBytes = 1ULL << 30;
hipError_t pool_alloc(void** p, size_t bytes, hipStream_t st);

// LDS one workgroup may use on the current device (bytes).
size_t max_lds_per_group();
// Lets `kernel` launch with `bytes` of dynamic LDS (beyond the default limit where one applies).
template <typename F>
hipError_t allow_lds(F kernel, size_t bytes) {
  hipError_t e = hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) (void)hipGetLastError();  // not needed on every runtime: the launch reports real errors
  return hipSuccess;
}

// ---------------------------------------------------------------------------------------------
// Device helpers.
// ---------------------------------------------------------------------------------------------
constexpr uint64_t kPhi64 = 0x9E3779B97F4A7C15ULL;
constexpr uint64_t kSqrt2 = 0x6A09E667F3BCC909ULL;

// SplitMix64 output function (Steele, Lea, Flood; Stafford variant 13).
__host__ __device__ __forceinline__ uint64_t mix_a(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// MurmurHash3 fmix64 (Appleby).
__host__ __device__ __forceinline__ uint64_t mix_b(uint64_t k) {
  k ^= k >> 33;
  k *= 0xFF51AFD7ED558CCDULL;
  k ^= k >> 33;
  k *= 0xC4CEB9FE1A85EC53ULL;
  return k ^ (k >> 33);
}

// floor(z * m / 2^64) for m < 2^32, from two 32x32 products.
__device__ __forceinline__ uint32_t mulhi_u32(uint64_t z, uint32_t m) {
  uint64_t lo = (uint64_t)(uint32_t)z * m;
  uint64_t hi = (uint64_t)(uint32_t)(z >> 32) * m + (lo >> 32);
  return (uint32_t)(hi >> 32);
}

__device__ __forceinline__ void hash_key_u64(uint64_t key, uint64_t seed, uint64_t& hi, uint64_t& lo) {
  hi = mix_a(key ^ seed);
  lo = mix_b(key ^ seed ^ kSqrt2);
}

// The nb <= 8 bytes at p as a little-endian word, zero above them, from the aligned 8-byte words
// that hold them (an aligned word that holds one byte of a buffer lies inside the buffer's pages).
__device__ __forceinline__ uint64_t load_le_bytes(const uint8_t* p, uint32_t nb) {
  const uintptr_t addr = (uintptr_t)p;
  const uint64_t* w = (const uint64_t*)(addr & ~(uintptr_t)7);
  const uint32_t sh = (uint32_t)(addr & 7);
  uint64_t v = w[0] >> (8 * sh);
  if (sh && sh + nb > 8) v |= w[1] << (64 - 8 * sh);
  return nb >= 8 ? v : (v & ((1ULL << (8 * nb)) - 1));
}

// Byte string -> (hi, lo): two chains over little-endian 8-byte words (the last one zero-padded),
// finished with the length.
__device__ __forceinline__ void hash_key_str(const uint8_t* s, uint64_t len, uint64_t seed, uint64_t& hi,
                                             uint64_t& lo) {
  uint64_t a = seed, b = seed ^ kSqrt2;
  for (uint64_t i = 0; i < len; i += 8) {
    const uint64_t w = load_le_bytes(s + i, (uint32_t)min<uint64_t>(8, len - i));
    a = mix_a(a ^ w);
    b = mix_b(b ^ w);
  }
  hi = mix_a(a ^ len);
  lo = mix_b(b ^ len);
}

// 64-bit fingerprint of a key's code; the position hash sees the key only through it.
__device__ __forceinline__ uint64_t fingerprint(uint64_t hi, uint64_t lo) { return lo ^ mix_b(hi); }

// Seeded position hash h(x, s) in [0, m): w = (s + 1) * phi is the seed's Weyl value.
__device__ __forceinline__ uint32_t pos_hash(uint64_t f, uint64_t w, uint32_t m) {
  return mulhi_u32(mix_a(f ^ w), m);
}

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

// Select entry s (of kSelBlock ones) of a unary stream with nvals ones whose low 32 bits already hold
// the position of one number kSelBlock s: adds the distances to ones kSelBlock s + kSelSub k, k = 1,
// 2, 3 (kSelRelNone from 1023 on, 0 past the last one).  Reads at most 17 words of the stream.
__device__ __forceinline__ void sel_fill_entry(const uint64_t* __restrict__ un, uint64_t* __restrict__ sel,
                                               uint64_t s, uint64_t nvals) {
  const uint64_t a0 = sel[s] & 0xFFFFFFFFULL;
  uint64_t out = a0, word = a0 >> 6;
  const uint64_t last = (a0 + kSelRelNone) >> 6;  // words past it cannot hold a distance below 1023
  uint64_t x = un[word] & (~0ULL << (a0 & 63));
  uint32_t seen = 0;  // ones from a0 on before the bits of x
  for (uint32_t k = 1; k < kSelBlock / kSelSub; k++) {
    if (s * kSelBlock + k * kSelSub >= nvals) break;
    const uint32_t want = k * kSelSub;  // one a0 is the 0th
    uint64_t f = kSelRelNone;
    for (;;) {
      const uint32_t c = __popcll(x);
      if (seen + c > want) {
        const uint64_t rel = word * 64 + select_in_word(x, want - seen) - a0;
        f = rel < kSelRelNone ? rel : kSelRelNone;
        break;
      }
      if (word == last) break;
      seen += c;
      x = un[++word];
    }
    out |= f << (32 + 10 * (k - 1));
  }
  sel[s] = out;
}

// Bucket of a key: linear interpolation of the tabulated bucket function, scaled to B buckets.
__device__ __forceinline__ uint32_t bucket_of(uint64_t lo, const uint64_t* __restrict__ T, uint32_t B) {
  uint32_t k = (uint32_t)(lo >> 53);
  uint64_t f = (lo >> 21) & 0xFFFFFFFFULL;
  uint64_t t0 = T[k], t1 = T[k + 1];
  uint64_t y = t0 + (((t1 - t0) * f) >> 32);
  uint32_t b = (uint32_t)((y * B) >> 32);
  return b < B - 1 ? b : B - 1;
}

// Reads width (<= 64) bits at bit position pos of a word array (one zero word of slack follows
// every section, so the second word is always in bounds).
__device__ __forceinline__ uint64_t get_bits(const uint64_t* __restrict__ w, uint64_t pos, uint32_t width) {
  if (width == 0) return 0;
  uint64_t idx = pos >> 6;
  uint32_t sh = (uint32_t)(pos & 63);
  uint64_t v = w[idx] >> sh;
  if (sh + width > 64) v |= w[idx + 1] << (64 - sh);
  return width == 64 ? v : (v & ((1ULL << width) - 1));
}

__device__ __forceinline__ void put_bits_atomic(uint64_t* w, uint64_t pos, uint64_t v, uint32_t width) {
  if (width == 0) return;
  uint64_t idx = pos >> 6;
  uint32_t sh = (uint32_t)(pos & 63);
  atomicOr((unsigned long long*)&w[idx], (unsigned long long)(v << sh));
  if (sh + width > 64) atomicOr((unsigned long long*)&w[idx + 1], (unsigned long long)(v >> (64 - sh)));
}

// Expected table offset of partition j: floor(j * R / 2^32), R = floor(total * 2^32 / K).
__device__ __forceinline__ uint64_t expected_offset(uint64_t j, uint64_t R) {
  return (j * R >> 32) | (__umul64hi(j, R) << 32);
}

inline uint64_t expected_offset_host(uint64_t j, uint64_t R) {
  return (uint64_t)(((unsigned __int128)j * R) >> 32);
}

}  // namespace phobic
