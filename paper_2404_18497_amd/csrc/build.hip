// Construction of a PHOBIC MPHF on one MI355X (gfx950, wave64).
//
// Pipeline (one stream):
//   k_hash_count_*  : hash every key and histogram its partition j = mulhi(hi, K)
//   k_scan_offsets  : one workgroup: partition key offsets and table offsets (prefix sums, Sec. 4)
//   k_scatter_*     : hash again and scatter the 128-bit codes into their partition (order free)
//   k_bucket_sort   : one workgroup per partition: bucket of every key by the tabulated beta_eps
//                     (Sec. 3.1, Sec. 3.2, App. C.1), buckets ordered by size desc, index desc
//                     (Sec. 3, Sec. 5.1), key fingerprints rewritten in processing order
//   k_search        : one wavefront per partition: for each bucket the smallest pilot
//                     p = s m + d whose positions are distinct and free (Sec. 4, Sec. 4.2); the
//                     free-slot bitmap lives in LDS, the 64 lanes test 64 displacement windows of
//                     64 bits each at once, keys are streamed one at a time, ballot picks the
//                     smallest surviving displacement
//   k_encoder_stats : per encoder (bucket index i) the sums of v >> b for b = 0..32 and the maximum
//   host            : Kiely's Rice parameter or the Compact width per encoder, image layout
//   k_pack_*        : offsets, values, unary stream and select samples, remap (alpha < 1)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "phobic_internal.h"
#include "search.h"

namespace phobic {
namespace {

constexpr int kBlock = 256;

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// The start of a build in one launch: error words (4) and info words (8) cleared, and the n counters at
// cnt.
__global__ void k_build_clear(uint32_t* __restrict__ err, uint64_t* __restrict__ d64, uint32_t* __restrict__ cnt,
                              uint64_t n) {
  const uint64_t i0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i0 < 4) err[i0] = 0;
  if (i0 < 8) d64[i0] = 0;
  for (uint64_t i = i0; i < n; i += (uint64_t)gridDim.x * blockDim.x) cnt[i] = 0;
}

__global__ void k_fill_u64(uint64_t* __restrict__ p, uint64_t n, uint64_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// A fresh image of nw words: the header words hw[0..nh), the encoder words hw[nh..nh + ne) at word
// enc_at, zero elsewhere (the packing kernels OR their fields in afterwards).
__global__ void k_image_init(uint64_t* __restrict__ img, uint64_t nw, const uint64_t* __restrict__ hw, uint32_t nh,
                             uint64_t enc_at, uint32_t ne) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nw; i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t v = 0;
    if (i < nh)
      v = hw[i];
    else if (i - enc_at < ne)  // i >= enc_at >= nh here
      v = hw[nh + (i - enc_at)];
    img[i] = v;
  }
}

// out[c][r] = in[r][c] for an R x Cn array of u32, in 64 x 64 tiles staged through LDS so that both
// the reads (along a row of `in`) and the writes (along a row of `out`) are contiguous.
constexpr uint32_t kTile = 64;
__global__ __launch_bounds__(kTile * kTile / 16) void k_transpose_u32(const uint32_t* __restrict__ in, uint64_t R,
                                                                      uint64_t Cn, uint32_t* __restrict__ out) {
  __shared__ uint32_t tile[kTile][kTile + 1];
  const uint64_t tr = (R + kTile - 1) / kTile, tc = (Cn + kTile - 1) / kTile;
  for (uint64_t t = blockIdx.x; t < tr * tc; t += gridDim.x) {
    const uint64_t r0 = (t / tc) * kTile, c0 = (t % tc) * kTile;
    for (uint32_t y = threadIdx.y; y < kTile; y += kTile / 16) {
      const uint64_t r = r0 + y, c = c0 + threadIdx.x;
      tile[y][threadIdx.x] = (r < R && c < Cn) ? in[r * Cn + c] : 0u;
    }
    __syncthreads();
    for (uint32_t y = threadIdx.y; y < kTile; y += kTile / 16) {
      const uint64_t c = c0 + y, r = r0 + threadIdx.x;
      if (c < Cn && r < R) out[c * R + r] = tile[threadIdx.x][y];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// Hashing and partitioning
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_hash_count_u64(const uint64_t* __restrict__ keys, uint64_t n,
                                                           uint64_t seed, uint64_t K, uint32_t* __restrict__ cnt) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t hi = mix_a(keys[i] ^ seed);
    atomicAdd(&cnt[__umul64hi(hi, K)], 1u);
  }
}

__global__ __launch_bounds__(kBlock) void k_scatter_u64(const uint64_t* __restrict__ keys, uint64_t n, uint64_t seed,
                                                        uint64_t K, const uint64_t* __restrict__ off,
                                                        uint32_t* __restrict__ cur, ulonglong2* __restrict__ codes) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t hi, lo;
    hash_key_u64(keys[i], seed, hi, lo);
    uint64_t j = __umul64hi(hi, K);
    uint64_t pos = off[j] + atomicAdd(&cur[j], 1u);
    codes[pos] = make_ulonglong2(hi, lo);
  }
}

// Strings: hash once into a staging array (hashing costs more than re-reading 16 bytes).
__global__ __launch_bounds__(kBlock) void k_hash_count_str(const uint8_t* __restrict__ bytes,
                                                           const uint64_t* __restrict__ offs, uint64_t n, uint64_t seed,
                                                           uint64_t K, ulonglong2* __restrict__ stage,
                                                           uint32_t* __restrict__ cnt) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t a = offs[i], b = offs[i + 1];
    uint64_t hi, lo;
    hash_key_str(bytes + a, b - a, seed, hi, lo);
    stage[i] = make_ulonglong2(hi, lo);
    if (K) atomicAdd(&cnt[__umul64hi(hi, K)], 1u);  // K = 0: hashing only (the counts come later)
  }
}

__global__ __launch_bounds__(kBlock) void k_scatter_codes(const ulonglong2* __restrict__ stage, uint64_t n, uint64_t K,
                                                          const uint64_t* __restrict__ off, uint32_t* __restrict__ cur,
                                                          ulonglong2* __restrict__ codes) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    ulonglong2 c = stage[i];
    uint64_t j = __umul64hi(c.x, K);
    codes[off[j] + atomicAdd(&cur[j], 1u)] = c;
  }
}

// Few partitions (K <= kLdsParts): per-key global atomics on K counters contend, so each workgroup
// takes a contiguous chunk of the keys, counts its partitions in LDS, and adds or reserves them with
// one global atomic per (workgroup, partition); the scatter then ranks its keys in LDS inside the
// reserved ranges.  kCodes: the input is the staged (hi, lo) codes of strings.
constexpr uint32_t kLdsParts = 12288;

template <bool kCodes>
__device__ __forceinline__ ulonglong2 general_code(const uint64_t* keys, const ulonglong2* stage, uint64_t i,
                                                   uint64_t seed) {
  if (kCodes) return stage[i];
  uint64_t hi, lo;
  hash_key_u64(keys[i], seed, hi, lo);
  return make_ulonglong2(hi, lo);
}

template <bool kCodes, bool kScatter>
__global__ __launch_bounds__(kBlock) void k_general_lds(const uint64_t* __restrict__ keys,
                                                        const ulonglong2* __restrict__ stage, uint64_t n,
                                                        uint64_t per, uint64_t seed, uint64_t K,
                                                        const uint64_t* __restrict__ off, uint32_t* __restrict__ cnt,
                                                        ulonglong2* __restrict__ codes) {
  extern __shared__ __align__(16) uint32_t hist[];  // [K]
  const uint64_t c0 = blockIdx.x * per, c1 = min(n, c0 + per);
  for (uint32_t j = threadIdx.x; j < K; j += kBlock) hist[j] = 0;
  __syncthreads();
  for (uint64_t i = c0 + threadIdx.x; i < c1; i += kBlock)
    atomicAdd(&hist[__umul64hi(general_code<kCodes>(keys, stage, i, seed).x, K)], 1u);
  __syncthreads();
  // counting: add the chunk's counts; scatter: reserve the chunk's ranges (cnt is the cursor)
  for (uint32_t j = threadIdx.x; j < K; j += kBlock) {
    const uint32_t c = hist[j];
    if (c) {
      const uint32_t b = atomicAdd(&cnt[j], c);
      if (kScatter) hist[j] = b;
    }
  }
  if (!kScatter) return;
  __syncthreads();
  for (uint64_t i = c0 + threadIdx.x; i < c1; i += kBlock) {
    const ulonglong2 c = general_code<kCodes>(keys, stage, i, seed);
    const uint64_t j = __umul64hi(c.x, K);
    codes[off[j] + atomicAdd(&hist[j], 1u)] = c;
  }
}

__device__ __forceinline__ uint64_t table_slots(uint64_t nj, uint32_t an, uint32_t ad) {
  return an == ad ? nj : (nj * ad + an - 1) / an;
}

// One workgroup of 1024 threads: key offsets, table offsets, the counters reset for the scatter,
// and info = {max n_j, max m_j, total table size}.
__global__ __launch_bounds__(1024) void k_scan_offsets(uint32_t* __restrict__ cnt, uint64_t K, uint32_t an,
                                                       uint32_t ad, uint64_t* __restrict__ off,
                                                       uint64_t* __restrict__ toff, uint64_t* __restrict__ info) {
  __shared__ uint64_t sn[1024], sm[1024];
  __shared__ uint32_t mxn, mxm;
  const uint32_t t = threadIdx.x;
  if (t == 0) { mxn = 0; mxm = 0; }
  const uint64_t per = (K + 1023) / 1024;
  const uint64_t a = min(K, (uint64_t)t * per), b = min(K, a + per);
  uint64_t tn = 0, tm = 0;
  uint32_t lmx = 0, lmm = 0;
  for (uint64_t j = a; j < b; j++) {
    uint32_t c = cnt[j];
    uint64_t m = table_slots(c, an, ad);
    tn += c;
    tm += m;
    lmx = max(lmx, c);
    lmm = max(lmm, (uint32_t)min<uint64_t>(m, 0xFFFFFFFFULL));
  }
  sn[t] = tn;
  sm[t] = tm;
  __syncthreads();
  atomicMax(&mxn, lmx);
  atomicMax(&mxm, lmm);
  for (uint32_t d = 1; d < 1024; d <<= 1) {
    uint64_t vn = t >= d ? sn[t - d] : 0, vm = t >= d ? sm[t - d] : 0;
    __syncthreads();
    sn[t] += vn;
    sm[t] += vm;
    __syncthreads();
  }
  uint64_t pn = sn[t] - tn, pm = sm[t] - tm;
  for (uint64_t j = a; j < b; j++) {
    uint32_t c = cnt[j];
    off[j] = pn;
    toff[j] = pm;
    pn += c;
    pm += table_slots(c, an, ad);
    cnt[j] = 0;
  }
  if (t == 1023) {
    off[K] = sn[1023];
    toff[K] = sm[1023];
    info[0] = mxn;
    info[1] = mxm;
    info[2] = sm[1023];
  }
}

// ---------------------------------------------------------------------------------------------
// Bucket mapping and ordering, one workgroup (256 threads) per partition.
// LDS: cnt[nbpad] counts then start offsets, key[nbpad] sort keys (size << 16 | id), rec[n_j]
// per-key (bucket << 16 | rank in bucket).
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_bucket_sort(const ulonglong2* __restrict__ codes,
                                                        const uint64_t* __restrict__ off,
                                                        const uint64_t* __restrict__ T, uint32_t B, uint32_t nbpad,
                                                        uint64_t* __restrict__ sortedf, uint32_t* __restrict__ blist,
                                                        uint32_t* __restrict__ nbk, uint32_t* __restrict__ maxb) {
  extern __shared__ __align__(16) uint32_t lds[];
  uint32_t* cnt = lds;
  uint32_t* key = lds + nbpad;
  uint32_t* rec = lds + 2 * nbpad;
  __shared__ uint32_t part[kBlock];
  __shared__ uint32_t nonempty;
  const uint32_t tid = threadIdx.x;
  const uint64_t j = blockIdx.x;
  const uint64_t base = off[j];
  const uint32_t nj = (uint32_t)(off[j + 1] - base);

  for (uint32_t x = tid; x < nbpad; x += kBlock) cnt[x] = 0;
  if (tid == 0) nonempty = 0;
  __syncthreads();
  for (uint32_t i = tid; i < nj; i += kBlock) {
    uint32_t b = bucket_of(codes[base + i].y, T, B);
    uint32_t r = atomicAdd(&cnt[b], 1u);
    rec[i] = (b << 16) | r;
  }
  __syncthreads();
  uint32_t ne = 0;
  for (uint32_t x = tid; x < nbpad; x += kBlock) {
    uint32_t c = x < B ? cnt[x] : 0;
    key[x] = c ? ((c << 16) | x) : 0u;
    ne += c != 0;
  }
  atomicAdd(&nonempty, ne);
  __syncthreads();
  // bitonic sort of key[] into descending order: size first, then bucket index
  for (uint32_t k = 2; k <= nbpad; k <<= 1) {
    for (uint32_t s = k >> 1; s > 0; s >>= 1) {
      for (uint32_t x = tid; x < nbpad; x += kBlock) {
        uint32_t y = x ^ s;
        if (y > x) {
          uint32_t a = key[x], b = key[y];
          bool first_half = (x & k) == 0;
          if (first_half ? (a < b) : (a > b)) {
            key[x] = b;
            key[y] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  // exclusive prefix sum of the sizes in processing order -> start offset of each bucket
  const uint32_t ipt = (nbpad + kBlock - 1) / kBlock;
  const uint32_t x0 = min(nbpad, tid * ipt), x1 = min(nbpad, x0 + ipt);
  uint32_t local = 0;
  for (uint32_t x = x0; x < x1; x++) local += key[x] >> 16;
  part[tid] = local;
  __syncthreads();
  for (uint32_t d = 1; d < kBlock; d <<= 1) {
    uint32_t v = tid >= d ? part[tid - d] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  uint32_t run = part[tid] - local;
  const uint32_t nb = nonempty;
  for (uint32_t x = x0; x < x1; x++) {
    uint32_t kx = key[x];
    if (x < nb) {
      cnt[kx & 0xFFFF] = run;
      blist[j * B + x] = kx;
    }
    run += kx >> 16;
  }
  if (tid == 0) {
    nbk[j] = nb;
    if (nb) atomicMax(maxb, key[0] >> 16);
  }
  __syncthreads();
  for (uint32_t i = tid; i < nj; i += kBlock) {
    uint32_t r = rec[i];
    ulonglong2 c = codes[base + i];
    sortedf[base + cnt[r >> 16] + (r & 0xFFFF)] = fingerprint(c.x, c.y);
  }
}

// ---------------------------------------------------------------------------------------------
// Bucket mapping and ordering for wide partitions (more keys or buckets than one workgroup holds
// in LDS), one workgroup of kWideThreads per partition.  The per-bucket counts, then start
// offsets, live in a global row cnt[j B .. j B + B) (zero on entry) and every key's rank inside its
// bucket in rank[]; only the sort keys (size << 16 | bucket) of the nbpad buckets are in LDS.
// Keys of one partition are read twice (bucket and rank, then the scatter) and their buckets
// computed twice.  A bucket of 65536 or more keys sets the capacity bit.
// ---------------------------------------------------------------------------------------------
constexpr int kWideThreads = 1024;

__device__ __forceinline__ uint32_t load_l2_u32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kWideThreads) void k_bucket_sort_wide(const ulonglong2* __restrict__ codes,
                                                                   const uint64_t* __restrict__ off,
                                                                   const uint64_t* __restrict__ T, uint32_t B,
                                                                   uint32_t nbpad, uint32_t* __restrict__ cnt,
                                                                   uint32_t* __restrict__ rank,
                                                                   uint64_t* __restrict__ sortedf,
                                                                   uint32_t* __restrict__ blist,
                                                                   uint32_t* __restrict__ nbk, uint32_t* __restrict__ info) {
  extern __shared__ __align__(16) uint32_t lds[];
  uint32_t* key = lds;  // [nbpad]
  __shared__ uint32_t part[kWideThreads];
  __shared__ uint32_t nonempty, toolarge;
  const uint32_t tid = threadIdx.x;
  const uint64_t j = blockIdx.x;
  const uint64_t base = off[j];
  const uint32_t nj = (uint32_t)(off[j + 1] - base);
  uint32_t* row = cnt + j * B;
  if (tid == 0) {
    nonempty = 0;
    toolarge = 0;
  }
  for (uint32_t i = tid; i < nj; i += kWideThreads) {
    const uint32_t b = bucket_of(codes[base + i].y, T, B);
    rank[base + i] = atomicAdd(&row[b], 1u);
  }
  __threadfence();
  __syncthreads();
  uint32_t ne = 0, big = 0;
  for (uint32_t x = tid; x < nbpad; x += kWideThreads) {
    const uint32_t c = x < B ? load_l2_u32(&row[x]) : 0u;
    big |= c > 0xFFFFu;
    key[x] = c ? ((min(c, 0xFFFFu) << 16) | x) : 0u;
    ne += c != 0;
  }
  atomicAdd(&nonempty, ne);
  if (big) atomicOr(&toolarge, 1u);
  __syncthreads();
  if (toolarge) {
    if (tid == 0) atomicOr(&info[0], 1u << PHOBIC_E_CAPACITY);
    return;
  }
  // bitonic sort of key[] into descending order: size first, then bucket index
  for (uint32_t k = 2; k <= nbpad; k <<= 1) {
    for (uint32_t sd = k >> 1; sd > 0; sd >>= 1) {
      for (uint32_t x = tid; x < nbpad; x += kWideThreads) {
        const uint32_t y = x ^ sd;
        if (y > x) {
          const uint32_t a = key[x], b = key[y];
          if ((x & k) == 0 ? (a < b) : (a > b)) {
            key[x] = b;
            key[y] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  // exclusive prefix of the sizes in processing order: every bucket's start inside the partition
  const uint32_t ipt = (nbpad + kWideThreads - 1) / kWideThreads;
  const uint32_t x0 = min(nbpad, tid * ipt), x1 = min(nbpad, x0 + ipt);
  uint32_t local = 0;
  for (uint32_t x = x0; x < x1; x++) local += key[x] >> 16;
  part[tid] = local;
  __syncthreads();
  for (uint32_t d = 1; d < kWideThreads; d <<= 1) {
    const uint32_t v = tid >= d ? part[tid - d] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  uint32_t run = part[tid] - local;
  const uint32_t nb = nonempty;
  for (uint32_t x = x0; x < x1; x++) {
    const uint32_t kx = key[x];
    if (x < nb) {
      row[kx & 0xFFFF] = run;
      blist[j * B + x] = kx;
    }
    run += kx >> 16;
  }
  if (tid == 0) {
    nbk[j] = nb;
    if (nb) atomicMax(&info[1], key[0] >> 16);
  }
  __threadfence();
  __syncthreads();
  for (uint32_t i = tid; i < nj; i += kWideThreads) {
    const ulonglong2 c = codes[base + i];
    const uint32_t b = bucket_of(c.y, T, B);
    sortedf[base + load_l2_u32(&row[b]) + rank[base + i]] = fingerprint(c.x, c.y);
  }
}


// ---------------------------------------------------------------------------------------------
// Hash, partition, bucket and order, main path: coarse bins of G = 2^gshift consecutive partitions,
// and digits of 2^dshift consecutive coarse bins (at most kMaxDigits digits).
//
//   k_coarse_count    : R workgroups (rows), each over a contiguous range of keys, histogram the
//                       coarse bin c = j >> gshift of every key in LDS; the row and its digit sums are
//                       saved and the row is added to the bin totals with one atomic per bin
//   k_coarse_scan     : bin offsets (one workgroup)
//   k_digit_offsets   : per digit, the offset of every row's share (rows in order)
//   k_split_digits    : row r moves its keys to its share of every digit
//   k_split_bins      : each slice of a digit (the shares of g consecutive rows) moves its keys to
//                       its bins, reserving its chunk of every bin with one atomic
//   k_segment_sort    : one workgroup per coarse bin: partition of every key, bucket by the tabulated
//                       bucket function, ranks within (partition, bucket), buckets of every partition
//                       ordered by size desc and index desc, partition offsets, fingerprints written
//                       in processing order
// Both splits go tile by tile: a tile is grouped by destination in LDS, then written in runs, so
// every store of a wavefront lands in a few cache lines.  One split straight to the bins would
// scatter single 8-byte stores over R x C open lines, far more than L2 holds, and every store
// would leave the chip as a partial line.  No per-key global atomics.
// ---------------------------------------------------------------------------------------------
constexpr int kCoarseThreads = 1024;
constexpr uint32_t kCoarseGroups = 256;  // half the number of rows
constexpr uint32_t kMaxCoarse = 14336;   // bins held by the LDS histogram (56 KB)
constexpr uint32_t kMaxDigits = 256;     // destinations of one split (a byte each in LDS)
constexpr uint32_t kMaxSliceBins = 16384; // (slice, bin) starts of one digit (64 KB of LDS)
constexpr int kSplitThreads = 1024;      // workgroup of the splits
constexpr int kSegThreads = 512;
constexpr uint32_t kMaxG = 8;
constexpr size_t kSegLdsBytes = 61440;   // dynamic LDS of k_segment_sort
constexpr int kSegBatch = 6;             // items of a k_segment_sort thread loaded together (5 for
                                         // 16-byte records: their registers would spill)

template <bool kStr>
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_count(const uint64_t* __restrict__ keys,
                                                                 const uint8_t* __restrict__ bytes,
                                                                 const uint64_t* __restrict__ offs,
                                                                 ulonglong2* __restrict__ stage, uint64_t n,
                                                                 uint64_t per, uint64_t seed, uint64_t K,
                                                                 uint32_t gshift, uint32_t C, uint32_t dshift,
                                                                 uint32_t D, uint32_t* __restrict__ ccnt,
                                                                 uint32_t* __restrict__ hrow,
                                                                 uint32_t* __restrict__ drow) {
  extern __shared__ __align__(16) uint32_t hist[];
  const uint32_t tid = threadIdx.x;
  for (uint32_t x = tid; x < C; x += kCoarseThreads) hist[x] = 0;
  __syncthreads();
  const uint64_t a = min(n, (uint64_t)blockIdx.x * per), b = min(n, a + per);
  if (kStr) {
    for (uint64_t i = a + tid; i < b; i += kCoarseThreads) {
      uint64_t hi, lo;
      const uint64_t s0 = offs[i], s1 = offs[i + 1];
      hash_key_str(bytes + s0, s1 - s0, seed, hi, lo);
      stage[i] = make_ulonglong2(hi, lo);
      atomicAdd(&hist[(uint32_t)__umul64hi(hi, K) >> gshift], 1u);
    }
  } else {
    // four keys per thread and round, loaded unconditionally (index clamped to the range) so that
    // they are in flight together
    constexpr int kU = 4;
    for (uint64_t i0 = a + tid; i0 < b; i0 += (uint64_t)kU * kCoarseThreads) {
      uint64_t v[kU];
#pragma unroll
      for (int u = 0; u < kU; u++) v[u] = keys[min(i0 + (uint64_t)u * kCoarseThreads, b - 1)];
#pragma unroll
      for (int u = 0; u < kU; u++)
        if (i0 + (uint64_t)u * kCoarseThreads < b)
          atomicAdd(&hist[(uint32_t)__umul64hi(mix_a(v[u] ^ seed), K) >> gshift], 1u);
    }
  }
  __syncthreads();
  for (uint32_t x = tid; x < C; x += kCoarseThreads) {
    const uint32_t v = hist[x];
    hrow[(uint64_t)blockIdx.x * C + x] = v;
    if (v) atomicAdd(&ccnt[x], v);
  }
  for (uint32_t d = tid; d < D; d += kCoarseThreads) {
    const uint32_t c0 = d << dshift, c1 = min(C, (d + 1) << dshift);
    uint32_t s = 0;
    for (uint32_t c = c0; c < c1; c++) s += hist[c];
    drow[(uint64_t)blockIdx.x * D + d] = s;
  }
}

// cbase[c] = bins before c (cbase[C] = n); cur[c] = cbase[c] as the scatter cursor
__global__ __launch_bounds__(1024) void k_coarse_scan(const uint32_t* __restrict__ ccnt, uint32_t C,
                                                      uint64_t* __restrict__ cbase, uint32_t* __restrict__ cur) {
  __shared__ uint64_t sp[1024];
  const uint32_t t = threadIdx.x;
  const uint32_t per = (C + 1023) / 1024;
  const uint32_t a = min(C, t * per), b = min(C, a + per);
  uint64_t loc = 0;
  for (uint32_t x = a; x < b; x++) loc += ccnt[x];
  sp[t] = loc;
  __syncthreads();
  for (uint32_t d = 1; d < 1024; d <<= 1) {
    const uint64_t v = t >= d ? sp[t - d] : 0;
    __syncthreads();
    sp[t] += v;
    __syncthreads();
  }
  uint64_t run = sp[t] - loc;
  for (uint32_t x = a; x < b; x++) {
    cbase[x] = run;
    cur[x] = (uint32_t)run;
    run += ccnt[x];
  }
  if (t == 1023) cbase[C] = sp[1023];
}

// One workgroup per digit d (R <= 1024 rows): doff[d (R + 1) + r] = where row r's share of digit d
// starts, rows in order; doff[d (R + 1) + R] = where the digit ends.
__global__ __launch_bounds__(1024) void k_digit_offsets(const uint32_t* __restrict__ drow,
                                                        const uint64_t* __restrict__ cbase, uint32_t R,
                                                        uint32_t D, uint32_t dshift, uint32_t* __restrict__ doff) {
  __shared__ uint32_t sp[1024];
  const uint32_t t = threadIdx.x, d = blockIdx.x;
  const uint32_t v = t < R ? drow[(uint64_t)t * D + d] : 0u;
  sp[t] = v;
  __syncthreads();
  for (uint32_t k = 1; k < 1024; k <<= 1) {
    const uint32_t u = t >= k ? sp[t - k] : 0u;
    __syncthreads();
    sp[t] += u;
    __syncthreads();
  }
  const uint32_t base = (uint32_t)cbase[d << dshift];
  if (t < R) doff[(uint64_t)d * (R + 1) + t] = base + sp[t] - v;
  if (t == R - 1) doff[(uint64_t)d * (R + 1) + R] = base + sp[t];
}

// Elements of the splits: the u64 keys themselves (the bin is hashed again from the key), or the
// 128-bit codes of hashed strings (the bin comes from the high word).
template <typename E> struct SplitElem;
template <> struct SplitElem<uint64_t> {
  static constexpr int kPer = 6;  // elements per thread and tile (the LDS stays under 64 KB)
  __device__ static uint32_t bin(uint64_t v, uint64_t seed, uint64_t K, uint32_t gshift) {
    return (uint32_t)__umul64hi(mix_a(v ^ seed), K) >> gshift;
  }
};
template <> struct SplitElem<ulonglong2> {
  static constexpr int kPer = 3;
  __device__ static uint32_t bin(ulonglong2 v, uint64_t, uint64_t K, uint32_t gshift) {
    return (uint32_t)__umul64hi(v.x, K) >> gshift;
  }
};
template <typename E>
constexpr uint32_t split_tile() { return (uint32_t)kSplitThreads * SplitElem<E>::kPer; }
template <typename E>
constexpr size_t split_lds_bytes() {
  return split_tile<E>() * (sizeof(E) + 1) + 4 * kMaxDigits * sizeof(uint32_t);
}

static_assert(split_lds_bytes<uint64_t>() <= 65536 && split_lds_bytes<ulonglong2>() <= 65536, "split LDS");
static_assert(kMaxDigits == 4 * 64, "the tile scan takes four counts per lane of one wavefront");
static_assert(kSplitThreads >= (int)kMaxDigits, "thread q passes the start of destination q");

// LDS of a split: tile | dest byte per tile slot | count | tile base | write offset | cursor.
template <typename E>
struct SplitLds {
  E* tile;
  uint8_t* dst;
  uint32_t *cnt, *tb, *wofs, *gpos;
  __device__ explicit SplitLds(uint32_t* lds) {
    constexpr uint32_t T = split_tile<E>();
    tile = (E*)lds;
    cnt = (uint32_t*)(tile + T);
    tb = cnt + kMaxDigits;
    wofs = tb + kMaxDigits;
    gpos = wofs + kMaxDigits;
    dst = (uint8_t*)(gpos + kMaxDigits);
  }
};

// Workgroup barrier that orders LDS only: global loads stay in flight across it (a prefetch of the
// next tile survives) and stores are not waited for.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// threadIdx.x, hidden from the optimiser: addresses derived from it are then formed where they are
// used instead of being hoisted out of the tile loop, where a dozen 64-bit pointers would spill (and
// a reload from scratch makes every following store wait for all memory operations in flight).
__device__ __forceinline__ uint32_t opaque_tid() {
  uint32_t t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// The tile of the split that starts at t0 (< b), in registers: element i = r threads + tid; the
// slots past the end repeat the last element, so that every load is unconditional.
template <typename E>
__device__ __forceinline__ void split_load(const E* __restrict__ in, uint64_t t0, uint64_t b,
                                           E (&v)[SplitElem<E>::kPer]) {
  constexpr uint32_t T = split_tile<E>();
  const uint32_t last = (uint32_t)min<uint64_t>(T, b - t0) - 1;
  const uint32_t tid = opaque_tid();
#pragma unroll
  for (int r = 0; r < SplitElem<E>::kPer; r++) v[r] = in[t0 + min((uint32_t)r * kSplitThreads + tid, last)];
}

// One tile of tn elements held in v: grouped by destination in LDS, then written out in runs.
// `prefetch` runs once the tile sits in LDS, so that the next tile's loads overlap the writes.
template <typename E, bool kFull, class Dest, class Prefetch>
__device__ __forceinline__ void split_tile_step(const E (&v)[SplitElem<E>::kPer], uint32_t tn, uint32_t nd,
                                                Dest dest, SplitLds<E>& L, E* __restrict__ out, Prefetch prefetch) {
  constexpr int kPer = SplitElem<E>::kPer;
  const uint32_t tid = opaque_tid();
  uint32_t qr[kPer];  // destination | rank within the tile << 8
#pragma unroll
  for (int r = 0; r < kPer; r++) {
    const uint32_t q = dest(v[r]);
    qr[r] = q;
    if (kFull || (uint32_t)r * kSplitThreads + tid < tn) qr[r] |= atomicAdd(&L.cnt[q], 1u) << 8;
  }
  lds_barrier();
  if (tid < 64) {  // exclusive scan of the tile's counts by one wavefront, four per lane
    uint32_t c[4], s = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const uint32_t x = tid * 4 + k;
      c[k] = x < nd ? L.cnt[x] : 0u;
      s += c[k];
    }
    uint32_t inc = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(inc, d);
      if (tid >= (uint32_t)d) inc += y;
    }
    uint32_t run = inc - s;
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const uint32_t x = tid * 4 + k;
      if (x < nd) {
        L.tb[x] = run;
        L.wofs[x] = L.gpos[x] - run;  // modulo 2^32: slot s of destination x goes to wofs[x] + s
        L.gpos[x] += c[k];
        L.cnt[x] = 0;
      }
      run += c[k];
    }
  }
  lds_barrier();
#pragma unroll
  for (int r = 0; r < kPer; r++) {
    if (kFull || (uint32_t)r * kSplitThreads + tid < tn) {
      const uint32_t s = L.tb[qr[r] & 0xFF] + (qr[r] >> 8);
      L.tile[s] = v[r];
      L.dst[s] = (uint8_t)qr[r];
    }
  }
  prefetch();
  lds_barrier();
#pragma unroll
  for (int r = 0; r < kPer; r++) {
    const uint32_t s = (uint32_t)r * kSplitThreads + tid;
    if (kFull || s < tn) out[L.wofs[L.dst[s]] + s] = L.tile[s];
  }
  lds_barrier();
}

// Moves in[a, b) to out, destination q of element v = dest(v) < nd <= kMaxDigits: the elements with
// destination q go to out[start], out[start + 1], ... in the order they are met, where thread q
// passes its destination's start.  Every thread of the workgroup calls it.  The first tile's loads
// are issued before the starts go to LDS.  kPrefetch: the next tile is loaded while this one is
// written (for long ranges; it costs registers).
template <typename E, bool kPrefetch, class Dest>
__device__ __forceinline__ void split_range(const E* __restrict__ in, uint64_t a, uint64_t b, uint32_t nd,
                                            uint32_t start, Dest dest, SplitLds<E>& L, E* __restrict__ out) {
  constexpr int kPer = SplitElem<E>::kPer;
  constexpr uint32_t T = split_tile<E>();
  E v[kPer], w[kPer];
  if (a < b) split_load<E>(in, a, b, v);
  if (threadIdx.x < nd) {
    L.cnt[threadIdx.x] = 0;
    L.gpos[threadIdx.x] = start;
  }
  lds_barrier();
  for (uint64_t t0 = a; t0 < b; t0 += T) {
    const uint64_t t1 = t0 + T;
    if (!kPrefetch && t0 != a) split_load<E>(in, t0, b, v);
    auto prefetch = [&]() {
      if (kPrefetch && t1 < b) split_load<E>(in, t1, b, w);
    };
    if (t1 <= b)
      split_tile_step<E, true>(v, T, nd, dest, L, out, prefetch);
    else
      split_tile_step<E, false>(v, (uint32_t)(b - t0), nd, dest, L, out, prefetch);
    if (kPrefetch)
#pragma unroll
      for (int r = 0; r < kPer; r++) v[r] = w[r];
  }
}

// Row r (the count's workgroup r, keys [r per, (r + 1) per)) to its share of every digit.
template <typename E>
__global__ __launch_bounds__(kSplitThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_split_digits(
    const E* __restrict__ in, uint64_t n, uint64_t per, uint64_t seed, uint64_t K, uint32_t gshift, uint32_t dshift,
    uint32_t D, uint32_t R, const uint32_t* __restrict__ doff, E* __restrict__ out) {
  extern __shared__ __align__(16) uint32_t lds[];
  SplitLds<E> L(lds);
  const uint32_t r = blockIdx.x;
  const uint64_t a = min(n, (uint64_t)r * per), b = min(n, a + per);
  const uint32_t start = threadIdx.x < D ? doff[(uint64_t)threadIdx.x * (R + 1) + r] : 0u;
  split_range<E, true>(
      in, a, b, D, start, [=](const E& v) { return SplitElem<E>::bin(v, seed, K, gshift) >> dshift; }, L, out);
}

// One workgroup per digit d: spos[(d Q + s) 2^dshift + x] = where slice s of digit d (the shares of
// rows [s g, s g + g)) starts in bin c = d 2^dshift + x; slices in order.
__global__ __launch_bounds__(1024) void k_slice_offsets(const uint32_t* __restrict__ hrow,
                                                        const uint64_t* __restrict__ cbase, uint32_t C, uint32_t R,
                                                        uint32_t g, uint32_t Q, uint32_t dshift,
                                                        uint32_t* __restrict__ spos) {
  extern __shared__ __align__(16) uint32_t sv[];  // Q 2^dshift slice counts
  const uint32_t d = blockIdx.x, nb = 1u << dshift, tid = threadIdx.x;
  for (uint32_t e = tid; e < Q * nb; e += 1024) {
    const uint32_t sl = e >> dshift, c = (d << dshift) + (e & (nb - 1));
    const uint32_t r0 = sl * g, r1 = min(R, r0 + g);
    uint32_t v = 0;
    if (c < C)
      for (uint32_t r = r0; r < r1; r++) v += hrow[(uint64_t)r * C + c];
    sv[e] = v;
  }
  __syncthreads();
  for (uint32_t x = tid; x < nb; x += 1024) {
    const uint32_t c = (d << dshift) + x;
    uint32_t run = c < C ? (uint32_t)cbase[c] : 0u;
    for (uint32_t sl = 0; sl < Q; sl++) {
      spos[((uint64_t)d * Q + sl) * nb + x] = run;
      run += sv[sl * nb + x];
    }
  }
}

// Workgroup d Q + s: slice s of digit d to its 2^dshift bins.
template <typename E>
__global__ __launch_bounds__(kSplitThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_split_bins(
    const E* __restrict__ in, uint64_t seed, uint64_t K, uint32_t gshift, uint32_t dshift, uint32_t R, uint32_t g,
    uint32_t Q, const uint32_t* __restrict__ doff, const uint32_t* __restrict__ spos, E* __restrict__ out) {
  extern __shared__ __align__(16) uint32_t lds[];
  SplitLds<E> L(lds);
  const uint32_t d = blockIdx.x / Q, s = blockIdx.x % Q;
  const uint32_t r0 = s * g, r1 = min(R, r0 + g), nb = 1u << dshift;
  const uint64_t a = doff[(uint64_t)d * (R + 1) + r0], b = doff[(uint64_t)d * (R + 1) + r1];
  const uint32_t start = threadIdx.x < nb ? spos[(uint64_t)blockIdx.x * nb + threadIdx.x] : 0u;
  const uint32_t mask = nb - 1;
  split_range<E, false>(
      in, a, b, nb, start, [=](const E& v) { return SplitElem<E>::bin(v, seed, K, gshift) & mask; }, L, out);
}

// Descending bitonic sort of keys[0, n) (n a power of two; entries beyond are zero) by one wavefront
// in registers: element i = lane * E + r; sub-stages with distance below E stay inside a lane, the
// others exchange with lane ^ (distance / E).  No workgroup barrier.
template <int E>
__device__ __forceinline__ void wave_bitonic_desc(uint32_t* keys, uint32_t n, uint32_t lane) {
  constexpr uint32_t N = 64 * E;
  uint32_t v[E];
#pragma unroll
  for (int r = 0; r < E; r++) {
    const uint32_t i = lane * E + r;
    v[r] = i < n ? keys[i] : 0u;
  }
#pragma unroll
  for (uint32_t k = 2; k <= N; k <<= 1) {
#pragma unroll
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      if (j >= (uint32_t)E) {
        const uint32_t jl = j / E;
        const bool lower = (lane & jl) == 0;
#pragma unroll
        for (int r = 0; r < E; r++) {
          const bool desc = ((lane * E + r) & k) == 0;
          const uint32_t pv = __shfl_xor(v[r], (int)jl);
          v[r] = (lower == desc) ? max(v[r], pv) : min(v[r], pv);
        }
      } else {
#pragma unroll
        for (int r = 0; r < E; r++) {
          if ((r & j) == 0) {
            const bool desc = ((lane * E + r) & k) == 0;
            const uint32_t a = v[r], b = v[r ^ j];
            v[r] = desc ? max(a, b) : min(a, b);
            v[r ^ j] = desc ? min(a, b) : max(a, b);
          }
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < E; r++) {
    const uint32_t i = lane * E + r;
    if (i < n) keys[i] = v[r];
  }
}

// nbpad <= 512 (at most 8 keys per lane, so the registers do not limit the kernel's occupancy)
__device__ __forceinline__ void wave_sort_keys(uint32_t* keys, uint32_t nbpad, uint32_t lane) {
  if (nbpad <= 64) wave_bitonic_desc<1>(keys, nbpad, lane);
  else if (nbpad == 128) wave_bitonic_desc<2>(keys, nbpad, lane);
  else if (nbpad == 256) wave_bitonic_desc<4>(keys, nbpad, lane);
  else wave_bitonic_desc<8>(keys, nbpad, lane);
}

// One workgroup per coarse bin of up to kMaxG partitions.  info[0] |= error bits, info[1] = max
// bucket size, info[2] = max partition size.
//
// kIn = kInCodes: src holds (hi, lo) of one MPHF with K partitions; the partition is mulhi(hi, K).
// kIn = kInKeys: src holds the u64 keys of one MPHF, hashed here with `seed` (half the bytes of codes
// through the scatter and this kernel's reads).
// kIn = kInRecords (batches): src holds (fingerprint, lo with the partition's slot in the bin in its
// low three bits, which the bucket function never reads); partitions are global indices of the
// batch, this launch covers [jbase, jend), and kbase is the global index of its first key.
enum { kInCodes = 0, kInKeys = 1, kInRecords = 2 };
template <int kIn>
__global__ __launch_bounds__(kSegThreads) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_segment_sort(const void* __restrict__ src, uint64_t seed,
                                                              const uint64_t* __restrict__ cbase,
                                                              const uint64_t* __restrict__ T, uint32_t B,
                                                              uint32_t nbpad, uint32_t gshift, uint64_t K,
                                                              uint64_t jbase, uint64_t jend, uint64_t kbase,
                                                              uint32_t seg_cap, uint64_t* __restrict__ sortedf,
                                                              uint32_t* __restrict__ blist, uint32_t* __restrict__ nbk,
                                                              uint64_t* __restrict__ off, uint32_t* __restrict__ info,
                                                              ulonglong2* __restrict__ dbg) {
  constexpr int kItems = (int)((kSegLdsBytes / 4 + kSegThreads - 1) / kSegThreads);
  extern __shared__ __align__(16) uint32_t lds[];
  const uint32_t G = 1u << gshift;
  const uint32_t span = G * nbpad;
  uint32_t* cnt = lds;          // [G][nbpad]: counts, then start offsets inside the bin
  uint32_t* key = lds + span;   // [G][nbpad]: sort keys (size << 16 | bucket)
  uint32_t* rec = lds + 2 * span;  // per key: partition << 29 | bucket << 16 | rank
  __shared__ uint32_t part[kSegThreads];
  __shared__ uint32_t psize[kMaxG], nonempty[kMaxG];
  __shared__ uint64_t Ts[kTableIntervals + 1];  // the bucket-function table: LDS reads instead of
                                                // 64 scattered cache lines per wavefront load
  const uint32_t tid = threadIdx.x;
  const uint64_t c = blockIdx.x;
  const uint64_t j0 = jbase + (c << gshift);
  const uint32_t ghere = (uint32_t)min<uint64_t>(G, jend - j0);
  const uint64_t base = cbase[c];  // inside this launch's code array
  const uint32_t ns = (uint32_t)(cbase[c + 1] - base);
  if (ns > seg_cap) {  // the build fails; its partitions are left empty (the last one spans the bin)
    if (tid == 0) atomicOr(&info[0], 1u << PHOBIC_E_CAPACITY);
    if (tid < ghere) {
      off[j0 + tid] = kbase + base;
      nbk[j0 + tid] = 0;
    }
    if (tid == 0 && j0 + ghere == jend) off[jend] = kbase + base + ns;
    return;
  }
  for (uint32_t x = tid; x < span; x += kSegThreads) cnt[x] = 0;
  if (tid < kMaxG) { psize[tid] = 0; nonempty[tid] = 0; }
  for (uint32_t x = tid; x <= kTableIntervals; x += kSegThreads) Ts[x] = T[x];
  __syncthreads();
  // Items in batches of kSegBatch: the batch's loads are unconditional (the index clamped to the
  // bin), then its hashes and bucket-table reads, so each batch costs one round trip of each
  // instead of one per item; only the LDS ranking is guarded.
  constexpr int kBat = kIn == kInRecords ? kSegBatch - 1 : kSegBatch;
  uint64_t fp[kItems];
  const uint32_t nit = (ns + kSegThreads - 1) / kSegThreads;
  // the raw items of batch t0 (u64 keys: the key in .x), loaded unconditionally
  auto load_batch = [&](int t0, ulonglong2 (&cd)[kBat]) {
#pragma unroll
    for (int u = 0; u < kBat; u++) {
      const uint32_t i = min(tid + (uint32_t)(t0 + u) * kSegThreads, ns - 1);
      if (kIn == kInKeys) {
        cd[u].x = ((const uint64_t*)src)[base + i];
      } else {
        cd[u] = ((const ulonglong2*)src)[base + i];
      }
    }
  };
  // u64 keys and codes: the next batch is in flight while this one is hashed and ranked (records
  // load batch by batch: their registers would spill)
  constexpr bool kPre = kIn != kInRecords;
  ulonglong2 cd[kBat];
  if (kPre && nit) load_batch(0, cd);
#pragma unroll
  for (int t0 = 0; t0 < kItems; t0 += kBat) {
    if ((uint32_t)t0 >= nit) break;
    ulonglong2 nx[kBat];
    if (!kPre) load_batch(t0, cd);
    if (kPre && (uint32_t)(t0 + kBat) < nit) load_batch(t0 + kBat, nx);
    uint32_t pb[kBat];  // partition << 16 | bucket
#pragma unroll
    for (int u = 0; u < kBat; u++) {
      if (kIn == kInKeys) {
        uint64_t hi, lo;
        hash_key_u64(cd[u].x, seed, hi, lo);
        cd[u] = make_ulonglong2(hi, lo);
      }
      const uint32_t p = kIn == kInRecords ? (uint32_t)(cd[u].y & 7) : (uint32_t)(__umul64hi(cd[u].x, K) - j0);
      pb[u] = (p << 16) | bucket_of(cd[u].y, Ts, B);
    }
#pragma unroll
    for (int u = 0; u < kBat; u++) {
      const uint32_t i = tid + (uint32_t)(t0 + u) * kSegThreads;
      if (t0 + u < kItems && i < ns) {
        const uint32_t p = pb[u] >> 16, b = pb[u] & 0xFFFF;
        const uint32_t r = atomicAdd(&cnt[p * nbpad + b], 1u);
        rec[i] = (p << 29) | (b << 16) | r;
        fp[t0 + u] = kIn == kInRecords ? (uint64_t)cd[u].x : fingerprint(cd[u].x, cd[u].y);
      }
    }
    if (kPre)
#pragma unroll
      for (int u = 0; u < kBat; u++) cd[u] = nx[u];
  }
  __syncthreads();
  for (uint32_t x = tid; x < span; x += kSegThreads) {
    const uint32_t p = x / nbpad, xb = x % nbpad;
    const uint32_t v = xb < B ? cnt[x] : 0;
    key[x] = v ? ((v << 16) | xb) : 0u;
    if (v) {
      atomicAdd(&psize[p], v);
      atomicAdd(&nonempty[p], 1u);
    }
  }
  __syncthreads();
  // every partition's nbpad keys into descending order (size, then bucket index)
  if (nbpad <= 512) {  // wavefront p sorts partition p (G <= kMaxG <= the workgroup's wavefronts)
    if ((tid >> 6) < G) wave_sort_keys(key + (tid >> 6) * nbpad, nbpad, tid & 63);
    __syncthreads();
  } else {  // many buckets: bitonic over the whole workgroup
    for (uint32_t k = 2; k <= nbpad; k <<= 1) {
      for (uint32_t sd = k >> 1; sd > 0; sd >>= 1) {
        for (uint32_t x = tid; x < span; x += kSegThreads) {
          const uint32_t y = x ^ sd;
          if (y > x) {
            const uint32_t a = key[x], b = key[y];
            // direction from the index inside the partition's block, so every block ends descending
            if (((x & (nbpad - 1)) & k) == 0 ? (a < b) : (a > b)) {
              key[x] = b;
              key[y] = a;
            }
          }
        }
        __syncthreads();
      }
    }
  }
  // exclusive prefix of the sizes over [G][nbpad] in order = start of every bucket inside the bin
  const uint32_t ipt = (span + kSegThreads - 1) / kSegThreads;
  const uint32_t x0 = min(span, tid * ipt), x1 = min(span, x0 + ipt);
  uint32_t local = 0;
  for (uint32_t x = x0; x < x1; x++) local += key[x] >> 16;
  part[tid] = local;
  __syncthreads();
  for (uint32_t d = 1; d < kSegThreads; d <<= 1) {
    const uint32_t v = tid >= d ? part[tid - d] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  uint32_t run = part[tid] - local;
  for (uint32_t x = x0; x < x1; x++) {
    const uint32_t kx = key[x];
    const uint32_t p = x / nbpad, xb = x % nbpad;
    if (xb < nonempty[p]) {
      cnt[p * nbpad + (kx & 0xFFFF)] = run;
      blist[(j0 + p) * B + xb] = kx;
    }
    run += kx >> 16;
  }
  if (tid < ghere) {
    uint32_t st = 0;
    for (uint32_t q = 0; q < tid; q++) st += psize[q];
    off[j0 + tid] = kbase + base + st;
    nbk[j0 + tid] = nonempty[tid];
    atomicMax(&info[1], key[tid * nbpad] >> 16);
    atomicMax(&info[2], psize[tid]);
  }
  if (tid == 0 && j0 + ghere == jend) off[jend] = kbase + base + ns;
  __syncthreads();
  // destinations inside the bin, then the fingerprints through LDS (free again) in rounds of
  // kSegLdsBytes / 8 so that the stores to global memory are contiguous
  // (two 16-bit destinations per register: a bin holds fewer than 2^16 keys)
  uint32_t dst2[(kItems + 1) / 2];
#pragma unroll
  for (int t = 0; t < (kItems + 1) / 2; t++) dst2[t] = 0;
#pragma unroll
  for (int t = 0; t < kItems; t++) {
    const uint32_t i = tid + t * kSegThreads;
    if (i < ns) {
      const uint32_t r = rec[i];
      const uint32_t d = cnt[(r >> 29) * nbpad + ((r >> 16) & 0x1FFF)] + (r & 0xFFFF);
      dst2[t / 2] |= d << (16 * (t & 1));
      if (dbg) {
        ulonglong2 cd;
        if (kIn == kInKeys) {
          uint64_t hi, lo;
          hash_key_u64(((const uint64_t*)src)[base + i], seed, hi, lo);
          cd = make_ulonglong2(hi, lo);
        } else {
          cd = ((const ulonglong2*)src)[base + i];
        }
        dbg[kbase + base + d] = cd;
      }
    }
  }
  __syncthreads();
  uint64_t* stage = (uint64_t*)lds;
  constexpr uint32_t kRound = (uint32_t)(kSegLdsBytes / 8);
  for (uint32_t q0 = 0; q0 < ns; q0 += kRound) {
#pragma unroll
    for (int t = 0; t < kItems; t++) {
      const uint32_t i = tid + t * kSegThreads;
      const uint32_t d = (dst2[t / 2] >> (16 * (t & 1))) & 0xFFFFu;
      if (i < ns && d - q0 < kRound) stage[d - q0] = fp[t];
    }
    __syncthreads();
    const uint32_t cntq = min(kRound, ns - q0);
    for (uint32_t x = tid; x < cntq; x += kSegThreads) sortedf[kbase + base + q0 + x] = stage[x];
    __syncthreads();
  }
}

// Table offsets for alpha < 1 from the key offsets: toff[j] = sum of ceil(n_j' den / num), j' < j;
// info[3] = max table size, tot[0] = total.
__global__ __launch_bounds__(1024) void k_table_offsets(const uint64_t* __restrict__ off, uint64_t K, uint32_t an,
                                                        uint32_t ad, uint64_t* __restrict__ toff,
                                                        uint32_t* __restrict__ info, uint64_t* __restrict__ tot) {
  __shared__ uint64_t sp[1024];
  __shared__ uint32_t mx;
  const uint32_t t = threadIdx.x;
  if (t == 0) mx = 0;
  const uint64_t per = (K + 1023) / 1024;
  const uint64_t a = min(K, (uint64_t)t * per), b = min(K, a + per);
  uint64_t loc = 0;
  uint32_t lmx = 0;
  for (uint64_t j = a; j < b; j++) {
    const uint64_t m = table_slots(off[j + 1] - off[j], an, ad);
    loc += m;
    lmx = max(lmx, (uint32_t)min<uint64_t>(m, 0xFFFFFFFFULL));
  }
  sp[t] = loc;
  __syncthreads();
  atomicMax(&mx, lmx);
  for (uint32_t d = 1; d < 1024; d <<= 1) {
    const uint64_t v = t >= d ? sp[t - d] : 0;
    __syncthreads();
    sp[t] += v;
    __syncthreads();
  }
  uint64_t run = sp[t] - loc;
  for (uint64_t j = a; j < b; j++) {
    toff[j] = run;
    run += table_slots(off[j + 1] - off[j], an, ad);
  }
  if (t == 1023) {
    toff[K] = sp[1023];
    tot[0] = sp[1023];
    info[3] = mx;
  }
}

// ---------------------------------------------------------------------------------------------
// Interleaved coding
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// The encoders' values go through the statistics and the packing in chunks of kPackChunk.
constexpr int kPackThreads = 1024;
constexpr int kPackItems = 4;
constexpr uint32_t kPackChunk = kPackThreads * kPackItems;
// k_encoder_stats: one chunk per workgroup, so that its byte counters (at most kPackChunk / kBlock
// per thread) and its 16-bit count fields (at most kPackChunk) cannot overflow.
static_assert(kPackChunk / kBlock <= 255 && kPackChunk < 65536, "count fields of k_encoder_stats");

// Workgroup (c, i) reads chunk c of encoder i (j in [c kPackChunk, (c + 1) kPackChunk), gridDim.x
// chunks): shsum[i * 33 + b] += sum_j (v_ij >> b), vmax[i] = max(vmax[i], max_j v_ij) (both start
// at zero, k_stats_init), and the chunk's bit counts c_k = #{j : bit k of v_ij is set} go to
// ccnt[(i gridDim.x + c) 32 + k].  Since v >> b = sum_{k >= b} bit_k(v) 2^(k - b), the counts give
// sum_j (v_ij >> b) = sum_{k >= b} c_k 2^(k - b) exactly, for any b, here and once the Rice
// parameters are known (k_chunk_carry).  A thread counts eight bits per add: byte t of cnt8[s]
// counts bit 8 t + s of its values.
__global__ __launch_bounds__(kBlock) void k_encoder_stats(const uint32_t* __restrict__ pilots, uint64_t K,
                                                          uint64_t* __restrict__ shsum, uint32_t* __restrict__ vmax,
                                                          uint32_t* __restrict__ ccnt) {
  __shared__ uint32_t wsum[kBlock / 64][16];
  __shared__ uint64_t cnt[32];
  __shared__ uint32_t mx;
  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, i = blockIdx.y;
  if (tid == 0) mx = 0;
  uint32_t cnt8[8];
#pragma unroll
  for (int t = 0; t < 8; t++) cnt8[t] = 0;
  uint32_t lmx = 0;
  const uint32_t* col = pilots + (uint64_t)i * K;
  {  // the thread's kPackChunk / kBlock values, all loads issued before the counting (clamped
     // index; a value past K counts as zero)
    constexpr int kPer = kPackChunk / kBlock;
    const uint64_t j0 = (uint64_t)blockIdx.x * kPackChunk + tid;
    uint32_t v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; u++) {
      const uint64_t jj = j0 + (uint64_t)u * kBlock;
      v[u] = col[jj < K ? jj : K - 1];
    }
#pragma unroll
    for (int u = 0; u < kPer; u++) {
      const uint32_t x = j0 + (uint64_t)u * kBlock < K ? v[u] : 0u;
      lmx = max(lmx, x);
#pragma unroll
      for (int t = 0; t < 8; t++) cnt8[t] += (x >> t) & 0x01010101u;
    }
  }
  // 16-bit fields: the counts of bits s and 16 + s (even bytes) and 8 + s and 24 + s (odd bytes); a
  // field sums at most kPackChunk < 2^16 values over the workgroup
#pragma unroll
  for (int t = 0; t < 8; t++) {
    const uint32_t ev = wave_sum_u32(cnt8[t] & 0x00FF00FFu), od = wave_sum_u32((cnt8[t] >> 8) & 0x00FF00FFu);
    if (lane == 0) {
      wsum[wave][2 * t] = ev;
      wsum[wave][2 * t + 1] = od;
    }
  }
  __syncthreads();
  atomicMax(&mx, lmx);
  if (tid < 32) {  // c_k for k = tid: byte k >> 3 of the counters of bit k & 7
    const uint32_t t = tid & 7, byte = tid >> 3;
    uint32_t f = 0;
    for (int w = 0; w < kBlock / 64; w++) f += wsum[w][2 * t + (byte & 1)];
    const uint32_t ck = (f >> (16 * (byte >> 1))) & 0xFFFFu;
    cnt[tid] = ck;
    ccnt[((uint64_t)i * gridDim.x + blockIdx.x) * 32 + tid] = ck;
  }
  __syncthreads();
  if (tid < 33) {
    uint64_t sb = 0;  // sum_{k >= b} c_k 2^(k - b) by Horner's rule from the top bit
    for (int k = 31; k >= (int)tid; k--) sb = 2 * sb + cnt[k];
    if (sb) atomicAdd((unsigned long long*)&shsum[(uint64_t)i * 33 + tid], (unsigned long long)sb);
  }
  if (tid == 0 && mx) atomicMax(&vmax[i], mx);
}

// Clears the statistics block of n words and sets the offset residue range at word mm_at to
// (LLONG_MAX, LLONG_MIN), the identities of the minimum and maximum taken by k_offset_stats.
__global__ void k_stats_init(uint64_t* __restrict__ st, uint64_t n, uint64_t mm_at) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    st[i] = i == mm_at ? (uint64_t)LLONG_MAX : (i == mm_at + 1 ? (uint64_t)LLONG_MIN : 0);
}

// Offset residues delta_j = toff[j] - E_j: minimum and maximum over j in [0, K].
__global__ __launch_bounds__(kBlock) void k_offset_stats(const uint64_t* __restrict__ toff, uint64_t K, uint64_t R,
                                                         long long* __restrict__ mm) {
  long long lmin = LLONG_MAX, lmax = LLONG_MIN;
  for (uint64_t jj = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; jj <= K; jj += (uint64_t)gridDim.x * blockDim.x) {
    long long d = (long long)(toff[jj] - expected_offset(jj, R));
    lmin = min(lmin, d);
    lmax = max(lmax, d);
  }
  __shared__ long long wmin[kBlock / 64], wmax[kBlock / 64];
  for (int o = 32; o > 0; o >>= 1) {
    lmin = min(lmin, (long long)__shfl_xor(lmin, o));
    lmax = max(lmax, (long long)__shfl_xor(lmax, o));
  }
  if ((threadIdx.x & 63) == 0) {
    wmin[threadIdx.x >> 6] = lmin;
    wmax[threadIdx.x >> 6] = lmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {  // one pair of atomics per workgroup
    for (int w = 1; w < kBlock / 64; w++) {
      lmin = min(lmin, wmin[w]);
      lmax = max(lmax, wmax[w]);
    }
    atomicMin(&mm[0], lmin);
    atomicMax(&mm[1], lmax);
  }
}

__global__ __launch_bounds__(kBlock) void k_pack_offsets(const uint64_t* __restrict__ toff, uint64_t K, uint64_t R,
                                                         long long dmin, uint32_t woff, uint64_t* __restrict__ sec) {
  for (uint64_t jj = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; jj <= K; jj += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t u = (uint64_t)((long long)(toff[jj] - expected_offset(jj, R)) - dmin);
    put_bits_atomic(sec, jj * woff, u, woff);
  }
}

// Rice: the unary start of every chunk, carry[i nch + c] = ubase_i + the unary length of chunks
// c' < c of encoder i, where a chunk's length is sum_j ((v_ij >> w_i) + 1), from its bit counts.
// One workgroup per Rice encoder (i0 + blockIdx.x; the encoders below i0 are Compact), nch chunks of
// kPackChunk values.
__global__ __launch_bounds__(kBlock) void k_chunk_carry(const uint32_t* __restrict__ ccnt, uint64_t K, uint64_t nch,
                                                        const uint64_t* __restrict__ enc,
                                                        const uint64_t* __restrict__ ubase,
                                                        uint64_t* __restrict__ carry, uint32_t i0) {
  __shared__ uint64_t part[kBlock / 64];
  const uint32_t tid = threadIdx.x, ln = tid & 63, i = i0 + blockIdx.x;  // Rice encoders i >= i0
  const int w = (int)(enc[i] & 0xFF);
  uint64_t run = ubase[i];
  for (uint64_t c0 = 0; c0 < nch; c0 += kBlock) {
    const uint64_t c = c0 + tid;
    uint64_t u = 0;
    if (c < nch) {
      const uint32_t* cc = ccnt + ((uint64_t)i * nch + c) * 32;
      for (int k = 31; k >= w; k--) u = 2 * u + cc[k];  // sum_j (v_ij >> w)
      u += min(K, (c + 1) * kPackChunk) - c * kPackChunk;
    }
    uint64_t incl = u;  // block inclusive scan
    for (int o = 1; o < 64; o <<= 1) {
      const uint64_t y = __shfl_up(incl, o);
      if (ln >= (uint32_t)o) incl += y;
    }
    if (ln == 63) part[tid >> 6] = incl;
    __syncthreads();
    uint64_t before = 0, total = 0;
    for (uint32_t x = 0; x < kBlock / 64; x++) {
      if (x < (tid >> 6)) before += part[x];
      total += part[x];
    }
    if (c < nch) carry[(uint64_t)i * nch + c] = run + before + incl - u;
    run += total;
    __syncthreads();
  }
}

// One workgroup of 1024 threads per chunk c and encoder i: low bits (or Compact values) at base_i + j w_i; for
// a Rice encoder (i >= ncompact when rice is set) the unary stream of q = v >> w_i (q zeros then a
// one), whose one for value t = (i - ncompact) K + j sits at ubase_i + sum_{j' < j} (q_j' + 1) + q_j,
// and the position of every 256th one in the select entries (their sub-sample distances are filled
// in afterwards, from the finished stream).
//
// A chunk's low bits (at most 4096 x 32 bits) and, when they fit, its unary bits (from the chunk's
// unary start, k_chunk_carry) are assembled in LDS and written out as whole words: plain stores for the
// words only this chunk touches, an atomic OR for its first and last word, which a neighbouring
// chunk or encoder may share.  A chunk whose unary run is too long for the buffer (a few huge
// pilots) sets its ones in global memory directly.
constexpr uint32_t kPackWords = kPackChunk / 2 + 2;  // 4096 fields of <= 32 bits, plus two partial words

__device__ __forceinline__ void lds_put_bits(uint64_t* buf, uint64_t rel, uint64_t v, uint32_t w) {
  const uint32_t idx = (uint32_t)(rel >> 6), sh = (uint32_t)(rel & 63);
  atomicOr((unsigned long long*)&buf[idx], (unsigned long long)(v << sh));
  if (sh + w > 64) atomicOr((unsigned long long*)&buf[idx + 1], (unsigned long long)(v >> (64 - sh)));
}


// Sub-sample distances of every select entry (the encoder wrote the samples), one thread per entry.
__global__ __launch_bounds__(kBlock) void k_sel_fill(const uint64_t* __restrict__ un, uint64_t* __restrict__ sel,
                                                     uint64_t nsel, uint64_t nvals) {
  for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < nsel; s += (uint64_t)gridDim.x * blockDim.x)
    sel_fill_entry(un, sel, s, nvals);
}

// Writes buf[0 .. last] to dst[first .. first + last]: interior words stored, the two end words ORed.
__device__ __forceinline__ void flush_words(const uint64_t* buf, uint64_t* __restrict__ dst, uint64_t first,
                                            uint32_t last, uint32_t tid) {
  for (uint32_t x = tid; x <= last; x += kPackThreads) {
    const uint64_t v = buf[x];
    if (x == 0 || x == last) {
      if (v) atomicOr((unsigned long long*)&dst[first + x], (unsigned long long)v);
    } else {
      dst[first + x] = v;
    }
  }
}

__global__ __launch_bounds__(kPackThreads) void k_pack_values(const uint32_t* __restrict__ pilots, uint64_t K,
                                                              const uint64_t* __restrict__ enc,
                                                              const uint64_t* __restrict__ carries, uint32_t rice_any,
                                                              uint32_t ncompact, uint64_t* __restrict__ data,
                                                              uint64_t* __restrict__ unary, uint64_t* __restrict__ sel) {
  __shared__ uint64_t part[kPackThreads / 64];
  __shared__ uint64_t chunk_total;
  __shared__ uint64_t dbuf[kPackWords];
  __shared__ uint64_t ubuf[kPackWords];
  const uint32_t tid = threadIdx.x, i = blockIdx.y;
  const bool rice = rice_any && i >= ncompact;
  const uint64_t e = enc[i];
  const uint32_t w = (uint32_t)(e & 0xFF);
  const uint64_t base = e >> 8;
  const uint32_t* col = pilots + (uint64_t)i * K;
  const uint64_t j0 = (uint64_t)blockIdx.x * kPackChunk;
  const uint64_t carry = rice ? carries[(uint64_t)i * gridDim.x + blockIdx.x] : 0;
  for (uint32_t x = tid; x < kPackWords; x += kPackThreads) {
    dbuf[x] = 0;
    ubuf[x] = 0;
  }
  const uint64_t jb = j0 + (uint64_t)tid * kPackItems;
  uint64_t v[kPackItems];
  uint64_t local = 0;
#pragma unroll
  for (int t = 0; t < kPackItems; t++) {
    v[t] = jb + t < K ? col[jb + t] : 0;
    if (jb + t < K) local += (v[t] >> w) + 1;
  }
  uint64_t incl = local;  // inclusive prefix of the unary lengths inside the wavefront
  if (rice) {
    // block exclusive scan of local
    const uint32_t ln = tid & 63;
    for (int o = 1; o < 64; o <<= 1) {
      uint64_t y = __shfl_up(incl, o);
      if (ln >= (uint32_t)o) incl += y;
    }
    if (ln == 63) part[tid >> 6] = incl;
    __syncthreads();
    if (tid < 64) {
      uint64_t pv = tid < kPackThreads / 64 ? part[tid] : 0;
      uint64_t pi = pv;
      for (int o = 1; o < 64; o <<= 1) {
        uint64_t y = __shfl_up(pi, o);
        if (tid >= (uint32_t)o) pi += y;
      }
      if (tid < kPackThreads / 64) part[tid] = pi - pv;
      if (tid == kPackThreads / 64 - 1) chunk_total = pi;
    }
  }
  __syncthreads();  // buffers cleared; scan results visible
  const uint64_t ctot = rice ? chunk_total : 0;
  uint64_t excl = rice ? carry + part[tid >> 6] + (incl - local) : 0;
  const uint64_t jend = min(K, j0 + kPackChunk);
  const uint64_t d_first = (base + j0 * w) >> 6;
  const uint64_t u_first = carry >> 6;
  const bool u_lds = ctot == 0 || ((carry + ctot - 1) >> 6) - u_first < kPackWords;
#pragma unroll
  for (int t = 0; t < kPackItems; t++) {
    const uint64_t jj = jb + t;
    if (jj < K) {
      const uint64_t q = v[t] >> w;
      if (w) lds_put_bits(dbuf, base + jj * w - d_first * 64, v[t] & ((1ULL << w) - 1), w);
      if (rice) {
        const uint64_t pos = excl + q;
        if (u_lds)
          atomicOr((unsigned long long*)&ubuf[(pos >> 6) - u_first], 1ULL << (pos & 63));
        else
          atomicOr((unsigned long long*)&unary[pos >> 6], 1ULL << (pos & 63));
        const uint64_t t_glob = (uint64_t)(i - ncompact) * K + jj;
        if ((t_glob & (kSelBlock - 1)) == 0) sel[t_glob / kSelBlock] = pos;
        excl = pos + 1;
      }
    }
  }
  __syncthreads();
  if (w) flush_words(dbuf, data, d_first, (uint32_t)(((base + jend * w - 1) >> 6) - d_first), tid);
  if (rice && u_lds && ctot) flush_words(ubuf, unary, u_first, (uint32_t)(((carry + ctot - 1) >> 6) - u_first), tid);
}

// ---------------------------------------------------------------------------------------------
// Remap for alpha < 1.  Table positions g >= n that hold a key, ascending, are paired with the
// free positions < n, ascending; entries of unoccupied g >= n repeat the previous value (0 first).
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t low_mask(uint32_t b) { return b >= 64 ? ~0ULL : ((1ULL << b) - 1); }

// per word: free slots below n, occupied slots in [n, total)
__global__ __launch_bounds__(kBlock) void k_remap_count(const uint64_t* __restrict__ taken, uint64_t nw, uint64_t n,
                                                        uint64_t total, uint32_t* __restrict__ fc,
                                                        uint32_t* __restrict__ oc) {
  for (uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; w < nw; w += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t lo = w * 64;
    const uint64_t below = n > lo ? low_mask((uint32_t)min<uint64_t>(64, n - lo)) : 0;
    const uint64_t valid = total > lo ? low_mask((uint32_t)min<uint64_t>(64, total - lo)) : 0;
    const uint64_t t = taken[w];
    fc[w] = __popcll(~t & below);
    oc[w] = __popcll(t & valid & ~below);
  }
}

// Exclusive scans of fc and oc in place, in three steps: per-block sums (kScanBlock words per
// workgroup), a scan of the block sums by one workgroup, then each block's local scan plus its
// offset.
constexpr uint32_t kScanThreads = 1024, kScanPer = 8, kScanBlock = kScanThreads * kScanPer;

__global__ __launch_bounds__(kScanThreads) void k_pair_block_sums(const uint32_t* __restrict__ fc,
                                                                  const uint32_t* __restrict__ oc, uint64_t nw,
                                                                  uint64_t* __restrict__ bs) {
  __shared__ uint64_t wf[kScanThreads / 64], wo[kScanThreads / 64];
  const uint64_t w0 = (uint64_t)blockIdx.x * kScanBlock;
  uint64_t tf = 0, to = 0;
  for (uint32_t x = threadIdx.x; x < kScanBlock; x += kScanThreads) {
    const uint64_t w = w0 + x;
    if (w < nw) {
      tf += fc[w];
      to += oc[w];
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    tf += __shfl_xor(tf, o);
    to += __shfl_xor(to, o);
  }
  if ((threadIdx.x & 63) == 0) {
    wf[threadIdx.x >> 6] = tf;
    wo[threadIdx.x >> 6] = to;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t sf = 0, so = 0;
    for (uint32_t x = 0; x < kScanThreads / 64; x++) {
      sf += wf[x];
      so += wo[x];
    }
    bs[2 * (uint64_t)blockIdx.x] = sf;
    bs[2 * (uint64_t)blockIdx.x + 1] = so;
  }
}

// exclusive scan of the nb block sums (pairs) in place, one workgroup
__global__ __launch_bounds__(kScanThreads) void k_pair_scan_blocks(uint64_t* __restrict__ bs, uint64_t nb) {
  __shared__ uint64_t sf[kScanThreads], so[kScanThreads];
  const uint32_t t = threadIdx.x;
  const uint64_t per = (nb + kScanThreads - 1) / kScanThreads;
  const uint64_t a = min(nb, (uint64_t)t * per), b = min(nb, a + per);
  uint64_t tf = 0, to = 0;
  for (uint64_t x = a; x < b; x++) {
    tf += bs[2 * x];
    to += bs[2 * x + 1];
  }
  sf[t] = tf;
  so[t] = to;
  __syncthreads();
  for (uint32_t d = 1; d < kScanThreads; d <<= 1) {
    const uint64_t vf = t >= d ? sf[t - d] : 0, vo = t >= d ? so[t - d] : 0;
    __syncthreads();
    sf[t] += vf;
    so[t] += vo;
    __syncthreads();
  }
  uint64_t pf = sf[t] - tf, po = so[t] - to;
  for (uint64_t x = a; x < b; x++) {
    const uint64_t f = bs[2 * x], o = bs[2 * x + 1];
    bs[2 * x] = pf;
    bs[2 * x + 1] = po;
    pf += f;
    po += o;
  }
}

// block b: its kScanBlock words scanned locally (kScanPer consecutive words per thread) plus the
// block's offset from bs
__global__ __launch_bounds__(kScanThreads) void k_pair_apply(uint32_t* __restrict__ fc, uint32_t* __restrict__ oc,
                                                             uint64_t nw, const uint64_t* __restrict__ bs) {
  __shared__ uint64_t sf[kScanThreads], so[kScanThreads];
  const uint32_t t = threadIdx.x;
  const uint64_t w0 = (uint64_t)blockIdx.x * kScanBlock + (uint64_t)t * kScanPer;
  uint32_t f[kScanPer], o[kScanPer];
  uint64_t tf = 0, to = 0;
#pragma unroll
  for (uint32_t x = 0; x < kScanPer; x++) {
    const bool in = w0 + x < nw;
    f[x] = in ? fc[w0 + x] : 0u;
    o[x] = in ? oc[w0 + x] : 0u;
    tf += f[x];
    to += o[x];
  }
  sf[t] = tf;
  so[t] = to;
  __syncthreads();
  for (uint32_t d = 1; d < kScanThreads; d <<= 1) {
    const uint64_t vf = t >= d ? sf[t - d] : 0, vo = t >= d ? so[t - d] : 0;
    __syncthreads();
    sf[t] += vf;
    so[t] += vo;
    __syncthreads();
  }
  uint64_t pf = bs[2 * (uint64_t)blockIdx.x] + sf[t] - tf, po = bs[2 * (uint64_t)blockIdx.x + 1] + so[t] - to;
#pragma unroll
  for (uint32_t x = 0; x < kScanPer; x++) {
    if (w0 + x < nw) {
      fc[w0 + x] = (uint32_t)pf;
      oc[w0 + x] = (uint32_t)po;
    }
    pf += f[x];
    po += o[x];
  }
}

__global__ __launch_bounds__(kBlock) void k_remap_free(const uint64_t* __restrict__ taken, uint64_t nw, uint64_t n,
                                                       const uint32_t* __restrict__ fcx, uint32_t* __restrict__ freeslot) {
  for (uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; w < nw; w += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t lo = w * 64;
    if (lo >= n) continue;
    uint64_t f = ~taken[w] & low_mask((uint32_t)min<uint64_t>(64, n - lo));
    uint32_t r = fcx[w];
    while (f) {
      uint32_t b = (uint32_t)(__ffsll((long long)f) - 1);
      f &= f - 1;
      freeslot[r++] = (uint32_t)(lo + b);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_remap_fill(const uint64_t* __restrict__ taken, uint64_t n, uint64_t total,
                                                       const uint32_t* __restrict__ ocx,
                                                       const uint32_t* __restrict__ freeslot, uint32_t wr,
                                                       uint64_t* __restrict__ sec) {
  for (uint64_t g = n + blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < total; g += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t w = g >> 6;
    const uint32_t b = (uint32_t)(g & 63);
    uint64_t sel = low_mask(b + 1);  // bits <= b
    const uint64_t lo = w * 64;
    if (n > lo) sel &= ~low_mask((uint32_t)min<uint64_t>(64, n - lo));  // only bits >= n
    const uint64_t r = ocx[w] + __popcll(taken[w] & sel);  // occupied positions in [n, g]
    const uint64_t v = r ? freeslot[r - 1] : 0;
    put_bits_atomic(sec, (g - n) * wr, v, wr);
  }
}

// ---------------------------------------------------------------------------------------------
// Host orchestration
// ---------------------------------------------------------------------------------------------
uint32_t grid_for(uint64_t n, uint32_t block = kBlock, uint32_t cap = 256 * 32) {
  uint64_t g = (n + block - 1) / block;
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g, cap));
}

uint32_t bit_length(uint64_t v) { return v ? 64 - __builtin_clzll(v) : 0; }

uint32_t next_pow2(uint32_t v) {
  uint32_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Build scratch.  Device blocks (hipMalloc) and pinned host blocks (hipHostMalloc, for the small
// transfers between the phases) are grouped into workspaces that outlive the builds: a build leases
// one workspace per device (concurrent builds lease different ones), takes its buffers from the
// blocks in request order with a bump pointer, and returns the workspace once its stream is idle.
// Blocks are allocated only when a request does not fit (grow-only) and stay allocated until the
// process ends, so repeated builds of similar sizes allocate and free nothing.
struct WsBlock {
  void* p;
  size_t cap;
};
struct Workspace {
  int device = 0;
  std::vector<WsBlock> dev, host;
};
std::mutex g_ws_mu;
std::vector<Workspace*> g_ws_idle;

Workspace* lease_workspace(int device) {
  std::lock_guard<std::mutex> lock(g_ws_mu);
  for (size_t i = 0; i < g_ws_idle.size(); i++) {
    if (g_ws_idle[i]->device == device) {
      Workspace* w = g_ws_idle[i];
      g_ws_idle.erase(g_ws_idle.begin() + (ptrdiff_t)i);
      return w;
    }
  }
  Workspace* w = new Workspace();
  w->device = device;
  return w;
}

void return_workspace(Workspace* w) {
  std::lock_guard<std::mutex> lock(g_ws_mu);
  g_ws_idle.push_back(w);
}

// Runs f(i) for i in [0, n) on up to 16 host threads (sequentially for small n).
template <class F>
void parallel_for(uint64_t n, F f) {
  const uint32_t hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const uint32_t nt = n < 65536 ? 1 : hw;
  if (nt == 1) {
    for (uint64_t i = 0; i < n; i++) f(i);
    return;
  }
  std::vector<std::thread> th;
  const uint64_t per = (n + nt - 1) / nt;
  for (uint32_t t = 0; t < nt; t++) {
    const uint64_t a = t * per, b = std::min(n, a + per);
    if (a >= b) break;
    th.emplace_back([=, &f] {
      for (uint64_t i = a; i < b; i++) f(i);
    });
  }
  for (auto& x : th) x.join();
}

struct Scratch {
  hipStream_t st;
  Workspace* ws;
  size_t db = 0, doff = 0, hb = 0, hoff = 0;
  explicit Scratch(hipStream_t s) : st(s) {
    int d = 0;
    (void)hipGetDevice(&d);
    ws = lease_workspace(d);
  }
  template <class T>
  hipError_t get(T** p, uint64_t count) {
    void* q = nullptr;
    const hipError_t e = take(ws->dev, db, doff, std::max<uint64_t>(count, 1) * sizeof(T), false, &q);
    *p = (T*)q;
    return e;
  }
  // pinned host staging
  template <class T>
  hipError_t host(T** p, uint64_t count) {
    void* q = nullptr;
    const hipError_t e = take(ws->host, hb, hoff, std::max<uint64_t>(count, 1) * sizeof(T), true, &q);
    *p = (T*)q;
    return e;
  }
  // copies `count` values from src through pinned staging to the device address dst, on the stream
  template <class T>
  hipError_t upload(T* dst, const T* src, uint64_t count) {
    if (count == 0) return hipSuccess;
    T* stage = nullptr;
    hipError_t e = host(&stage, count);
    if (e != hipSuccess) return e;
    std::memcpy(stage, src, count * sizeof(T));
    return hipMemcpyAsync(dst, stage, count * sizeof(T), hipMemcpyHostToDevice, st);
  }
  ~Scratch() {
    (void)hipStreamSynchronize(st);  // nothing on the stream may still use the blocks
    return_workspace(ws);
  }

 private:
  static hipError_t take(std::vector<WsBlock>& bl, size_t& b, size_t& off, size_t bytes, bool pinned, void** out) {
    bytes = (bytes + 255) & ~(size_t)255;
    while (b < bl.size()) {
      if (off + bytes <= bl[b].cap) {
        *out = (char*)bl[b].p + off;
        off += bytes;
        return hipSuccess;
      }
      b++;
      off = 0;
    }
    const size_t cap = std::max(bytes, pinned ? ((size_t)4 << 20) : ((size_t)64 << 20));
    void* q = nullptr;
    const hipError_t e = pinned ? hipHostMalloc(&q, cap, hipHostMallocDefault) : hipMalloc(&q, cap);
    if (e != hipSuccess) return e;
    bl.push_back({q, cap});
    b = bl.size() - 1;
    off = bytes;
    *out = q;
    return hipSuccess;
  }
};

// Phase timing with events on the build's stream.  Events come from a per-thread, per-device pool
// and go back to it, so a build creates none once its thread has built before.
struct Timer {
  hipStream_t st;
  int dev = 0;
  std::vector<hipEvent_t> ev;
  static std::map<int, std::vector<hipEvent_t>>& pool() {
    static thread_local std::map<int, std::vector<hipEvent_t>> p;
    return p;
  }
  explicit Timer(hipStream_t s) : st(s) { (void)hipGetDevice(&dev); }
  void mark() {
    std::vector<hipEvent_t>& free = pool()[dev];
    hipEvent_t e = nullptr;
    if (!free.empty()) {
      e = free.back();
      free.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      return;
    }
    (void)hipEventRecord(e, st);
    ev.push_back(e);
  }
  double ms(size_t a, size_t b) const {
    float t = 0;
    if (b < ev.size() && hipEventElapsedTime(&t, ev[a], ev[b]) != hipSuccess) return 0;
    return b < ev.size() ? t : 0;
  }
  ~Timer() {
    std::vector<hipEvent_t>& free = pool()[dev];
    free.insert(free.end(), ev.begin(), ev.end());
  }
};

// Waits for the stream's work by polling it: a blocking wait can wake tens of microseconds after
// the work ends, and a build pays that at each of its host round trips.
hipError_t spin_sync(hipStream_t st) {
  for (;;) {
    const hipError_t e = hipStreamQuery(st);
    if (e != hipErrorNotReady) return e;
  }
}

void configure_pool_once() {
  static std::once_flag once;
  std::call_once(once, [] {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
      uint64_t thr = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
  });
}

enum class Src { U64, Str };

struct BuildInput {
  Src src;
  const uint64_t* keys;
  const uint8_t* bytes;
  const uint64_t* offs;
  uint64_t n;
};

// Bound on the largest bucket of a partition of about P keys: bucket 0 is the largest in
// expectation (the bucket function is convex), P x0 keys with x0 the hash range it covers, plus
// seven standard deviations.
static uint32_t bucket_size_bound(const phobic_params& prm, uint32_t B, uint64_t part_bound) {
  std::vector<uint64_t> T(kTableIntervals + 1);
  bucket_table(prm.lambda, prm.partition_size, prm.alpha_num, prm.alpha_den, prm.bucket_function, T.data());
  uint32_t k = 1;
  while (k < kTableIntervals && (unsigned __int128)T[k] * B < ((unsigned __int128)1 << 32)) k++;
  const double e0 = (double)prm.partition_size * (double)k / kTableIntervals;
  const double b = e0 + 7.0 * std::sqrt(e0) + 16.0;
  return (uint32_t)std::min<double>(b, (double)part_bound);
}

phobic_status build_impl(const BuildInput& in, const phobic_params* params, hipStream_t st, phobic_mphf** out,
                         uint64_t* part_offsets_out, uint64_t* part_codes_out, bool exact_sizes = false) {
  if (out) *out = nullptr;
  uint32_t B = 0;
  phobic_status vs = validate_params(params, &B);
  if (vs != PHOBIC_OK) return vs;
  if (B > kWideMaxBuckets)
    return fail(PHOBIC_E_CAPACITY, "B = ceil(P / lambda) = " + std::to_string(B) + " exceeds the device limit " +
                                       std::to_string(kWideMaxBuckets));
  if (in.n > 0 && ((in.src == Src::U64 && !in.keys) || (in.src == Src::Str && (!in.bytes || !in.offs))))
    return fail(PHOBIC_E_INVALID, "null key pointer");
  configure_pool_once();

  const phobic_params& prm = *params;
  const uint64_t n = in.n;
  const uint64_t K = num_partitions(n, prm.partition_size);
  const uint32_t an = prm.alpha_num, ad = prm.alpha_den;
  const uint64_t limit = prm.pilot_limit ? prm.pilot_limit : 0xFFFFFFFFULL;
  const bool keep = (prm.flags & PHOBIC_FLAG_KEEP_PILOTS) != 0;

  auto h = new phobic_mphf();
  struct Guard {
    phobic_mphf*& h;
    ~Guard() {
      if (h) phobic_free(h);
    }
  } guard{h};
  PHOBIC_HIP(hipGetDevice(&h->device));
  h->n = n;
  h->K = K;
  h->B = B;
  h->prm = prm;

  Scratch S(st);
  Timer tm(st);
  auto t_host0 = std::chrono::steady_clock::now();
  {
    phobic_status ts = upload_table(h, st);
    if (ts != PHOBIC_OK) return ts;
  }

  // ---- hash, partition, bucket, order -----------------------------------------------------------
  uint64_t *off, *toff = nullptr, *sortedf, *d64;
  uint32_t *blist, *nbk, *pilots, *err;  // err[0] error bits, [1] max bucket, [2] max n_j, [3] max m_j
  PHOBIC_HIP(S.get(&off, K + 1));
  PHOBIC_HIP(S.get(&sortedf, n));
  PHOBIC_HIP(S.get(&blist, K * B));
  PHOBIC_HIP(S.get(&nbk, K));
  PHOBIC_HIP(S.get(&err, 4));
  PHOBIC_HIP(S.get(&d64, 8));
  uint32_t* pilots_pm;  // partition-major rows from the search (every row written whole)
  if (keep) {
    PHOBIC_HIP(hipMalloc(&h->d_pilots, std::max<uint64_t>(1, K * B) * sizeof(uint32_t)));
    pilots_pm = h->d_pilots;
  } else {
    PHOBIC_HIP(S.get(&pilots_pm, K * B));
  }
  PHOBIC_HIP(S.get(&pilots, K * B));  // encoder-major copy for the encoders
  const uint32_t nbpad = next_pow2(B);
  const bool str = in.src == Src::Str;

  // coarse bins: the largest G = 2^gshift <= kMaxG whose bins (G P keys plus eight standard
  // deviations) fit the LDS of k_segment_sort
  int gshift = -1;
  uint32_t seg_cap = 0;
  for (int gs = 3; gs >= 0; gs--) {
    const double gp = (double)(1u << gs) * prm.partition_size;
    const int64_t cap = ((int64_t)kSegLdsBytes - 8 * (int64_t)(1u << gs) * nbpad) / 4;
    if (cap > 0 && gp + 8.0 * std::sqrt(gp) + 64.0 <= (double)cap) {
      gshift = gs;
      seg_cap = (uint32_t)cap;
      break;
    }
  }
  const uint64_t C = gshift >= 0 ? (K + (1ULL << gshift) - 1) >> gshift : 0;
  const bool coarse_path = gshift >= 0 && C <= kMaxCoarse && n < (1ULL << 32) && B <= kMaxBuckets;
  bool wide = false;  // partitions beyond the LDS of the per-partition workgroups (general path only)
  uint64_t* old_info;  // pinned: max n_j, max m_j, table total of the fallback path
  PHOBIC_HIP(S.host(&old_info, 3));
  old_info[0] = old_info[1] = old_info[2] = 0;

  if (coarse_path) {
    uint32_t *ccnt, *hrow, *drow, *doff, *spos, *cur;
    uint64_t* cbase;
    ulonglong2 *codes = nullptr, *stage = nullptr;
    // R = 2 ngrp rows of per keys each (the count and the first split run one workgroup per row)
    const uint32_t ngrp = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(kCoarseGroups, (n + 8191) / 8192));
    const uint32_t R = 2 * ngrp;
    const uint64_t per = std::max<uint64_t>(1, (n + R - 1) / R);  // at least 1: empty inputs divide by it
    uint32_t dshift = 0;
    while (((C + (1ULL << dshift) - 1) >> dshift) > kMaxDigits) dshift++;
    const uint32_t D = (uint32_t)((C + (1ULL << dshift) - 1) >> dshift);
    // With one bin per digit the first split already leaves every bin in place.  Otherwise the
    // second split takes slices of g rows' shares of a digit, about seven eighths of a tile, with
    // at most kMaxSliceBins (slice, bin) starts per digit.
    const bool two = dshift > 0;
    const uint64_t T = str ? split_tile<ulonglong2>() : split_tile<uint64_t>();
    uint32_t g = (uint32_t)std::min<uint64_t>(R, std::max<uint64_t>(1, T * 7 * D / (8 * per)));
    g = std::max<uint32_t>(g, (uint32_t)(((uint64_t)R << dshift) + kMaxSliceBins - 1) / kMaxSliceBins);
    const uint32_t Q = (R + g - 1) / g;
    PHOBIC_HIP(S.get(&ccnt, C));
    PHOBIC_HIP(S.get(&hrow, (uint64_t)R * C));
    PHOBIC_HIP(S.get(&drow, (uint64_t)R * D));
    PHOBIC_HIP(S.get(&doff, (uint64_t)D * (R + 1)));
    PHOBIC_HIP(S.get(&spos, ((uint64_t)D * Q) << dshift));
    PHOBIC_HIP(S.get(&cur, C));
    PHOBIC_HIP(S.get(&cbase, C + 1));
    uint64_t* kcodes = nullptr;  // u64 keys: the keys themselves travel through the splits
    if (str) {
      PHOBIC_HIP(S.get(&codes, n));
      PHOBIC_HIP(S.get(&stage, n));
    } else {
      PHOBIC_HIP(S.get(&kcodes, n));
    }
    const size_t hist_lds = C * sizeof(uint32_t);
    tm.mark();  // 0
    hipLaunchKernelGGL(k_build_clear, dim3(grid_for(std::max<uint64_t>(C, 8))), dim3(kBlock), 0, st, err, d64, ccnt, C);
    if (str)
      hipLaunchKernelGGL(k_coarse_count<true>, dim3(R), dim3(kCoarseThreads), hist_lds, st, in.keys, in.bytes,
                         in.offs, stage, n, per, prm.hash_seed, K, (uint32_t)gshift, (uint32_t)C, dshift, D, ccnt,
                         hrow, drow);
    else
      hipLaunchKernelGGL(k_coarse_count<false>, dim3(R), dim3(kCoarseThreads), hist_lds, st, in.keys, in.bytes,
                         in.offs, stage, n, per, prm.hash_seed, K, (uint32_t)gshift, (uint32_t)C, dshift, D, ccnt,
                         hrow, drow);
    tm.mark();  // 1
    hipLaunchKernelGGL(k_coarse_scan, dim3(1), dim3(1024), 0, st, ccnt, (uint32_t)C, cbase, cur);
    hipLaunchKernelGGL(k_digit_offsets, dim3(D), dim3(1024), 0, st, drow, cbase, R, D, dshift, doff);
    if (two)
      hipLaunchKernelGGL(k_slice_offsets, dim3(D), dim3(1024), ((size_t)Q << dshift) * sizeof(uint32_t), st, hrow,
                         cbase, (uint32_t)C, R, g, Q, dshift, spos);
    tm.mark();  // 2
    if (str) {
      hipLaunchKernelGGL(k_split_digits<ulonglong2>, dim3(R), dim3(kSplitThreads), split_lds_bytes<ulonglong2>(),
                         st, (const ulonglong2*)stage, n, per, prm.hash_seed, K, (uint32_t)gshift, dshift, D, R,
                         doff, codes);
      if (two) {
        hipLaunchKernelGGL(k_split_bins<ulonglong2>, dim3(D * Q), dim3(kSplitThreads),
                           split_lds_bytes<ulonglong2>(), st, (const ulonglong2*)codes, prm.hash_seed, K,
                           (uint32_t)gshift, dshift, R, g, Q, doff, spos, stage);
        std::swap(codes, stage);  // the bins are in `codes` from here on
      }
    } else {
      // the fingerprint array is free until the bucket sort and holds the digits in between
      uint64_t* mid = two ? sortedf : kcodes;
      hipLaunchKernelGGL(k_split_digits<uint64_t>, dim3(R), dim3(kSplitThreads), split_lds_bytes<uint64_t>(), st,
                         in.keys, n, per, prm.hash_seed, K, (uint32_t)gshift, dshift, D, R, doff, mid);
      if (two)
        hipLaunchKernelGGL(k_split_bins<uint64_t>, dim3(D * Q), dim3(kSplitThreads), split_lds_bytes<uint64_t>(),
                           st, (const uint64_t*)mid, prm.hash_seed, K, (uint32_t)gshift, dshift, R, g, Q, doff, spos,
                           kcodes);
    }
    tm.mark();  // 3
    if (str)
      hipLaunchKernelGGL(k_segment_sort<kInCodes>, dim3((uint32_t)C), dim3(kSegThreads), kSegLdsBytes, st,
                         (const void*)codes, prm.hash_seed, cbase, h->d_table, B, nbpad, (uint32_t)gshift, K,
                         (uint64_t)0, K, (uint64_t)0, seg_cap, sortedf, blist, nbk, off, err,
                         (ulonglong2*)part_codes_out);
    else
      hipLaunchKernelGGL(k_segment_sort<kInKeys>, dim3((uint32_t)C), dim3(kSegThreads), kSegLdsBytes, st,
                         (const void*)kcodes, prm.hash_seed, cbase, h->d_table, B, nbpad, (uint32_t)gshift, K,
                         (uint64_t)0, K, (uint64_t)0, seg_cap, sortedf, blist, nbk, off, err,
                         (ulonglong2*)part_codes_out);
    if (an != ad) {
      PHOBIC_HIP(S.get(&toff, K + 1));
      hipLaunchKernelGGL(k_table_offsets, dim3(1), dim3(1024), 0, st, off, K, an, ad, toff, err, d64);
    } else {
      toff = off;
    }
    tm.mark();  // 4
    PHOBIC_HIP(hipGetLastError());
  } else {
    // general path for very many partitions: per-key global atomics
    uint32_t* cnt;
    uint64_t* dinfo;
    ulonglong2 *codes, *stage = nullptr;
    PHOBIC_HIP(S.get(&cnt, K + 1));
    PHOBIC_HIP(S.get(&toff, K + 1));
    PHOBIC_HIP(S.get(&dinfo, 8));
    PHOBIC_HIP(S.get(&codes, n));
    if (str) PHOBIC_HIP(S.get(&stage, n));
    tm.mark();  // 0
    hipLaunchKernelGGL(k_build_clear, dim3(grid_for(std::max<uint64_t>(K + 1, 8))), dim3(kBlock), 0, st, err, d64,
                       cnt, K + 1);
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, dinfo, (uint64_t)8, (uint64_t)0);
    const bool lds_parts = K <= kLdsParts;  // few partitions: LDS counts per chunk of keys
    const uint32_t chunks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(2048, (n + 8191) / 8192));
    const uint64_t per = std::max<uint64_t>(1, (n + chunks - 1) / chunks);
    if (str)  // strings are hashed once into the staging array
      hipLaunchKernelGGL(k_hash_count_str, dim3(grid_for(n)), dim3(kBlock), 0, st, in.bytes, in.offs, n,
                         prm.hash_seed, lds_parts ? (uint64_t)0 : K, stage, cnt);
    if (lds_parts && str)
      hipLaunchKernelGGL((k_general_lds<true, false>), dim3(chunks), dim3(kBlock), K * sizeof(uint32_t), st,
                         in.keys, stage, n, per, prm.hash_seed, K, off, cnt, codes);
    else if (lds_parts)
      hipLaunchKernelGGL((k_general_lds<false, false>), dim3(chunks), dim3(kBlock), K * sizeof(uint32_t), st,
                         in.keys, stage, n, per, prm.hash_seed, K, off, cnt, codes);
    else if (!str)
      hipLaunchKernelGGL(k_hash_count_u64, dim3(grid_for(n)), dim3(kBlock), 0, st, in.keys, n, prm.hash_seed, K, cnt);
    tm.mark();  // 1
    hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(1024), 0, st, cnt, K, an, ad, off, toff, dinfo);
    tm.mark();  // 2
    PHOBIC_HIP(hipGetLastError());
    PHOBIC_HIP(hipMemcpyAsync(old_info, dinfo, 3 * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    PHOBIC_HIP(hipStreamSynchronize(st));
    // wide partitions: bucketing with global counts and a search whose bucket list and pilots stay
    // in global memory (the LDS keeps the slot bitmaps and the current bucket's positions only)
    wide = B > kMaxBuckets || old_info[0] > kMaxPartitionKeys || old_info[1] > kMaxTableSlots;
    if (wide && old_info[1] >= kWideMaxTableSlots)
      return fail(PHOBIC_E_CAPACITY, "a partition needs " + std::to_string(old_info[1]) +
                                         " slots; the device path holds fewer than " +
                                         std::to_string(kWideMaxTableSlots));
    if (lds_parts && str)
      hipLaunchKernelGGL((k_general_lds<true, true>), dim3(chunks), dim3(kBlock), K * sizeof(uint32_t), st, in.keys,
                         stage, n, per, prm.hash_seed, K, off, cnt, codes);
    else if (lds_parts)
      hipLaunchKernelGGL((k_general_lds<false, true>), dim3(chunks), dim3(kBlock), K * sizeof(uint32_t), st,
                         in.keys, stage, n, per, prm.hash_seed, K, off, cnt, codes);
    else if (!str)
      hipLaunchKernelGGL(k_scatter_u64, dim3(grid_for(n)), dim3(kBlock), 0, st, in.keys, n, prm.hash_seed, K, off,
                         cnt, codes);
    else
      hipLaunchKernelGGL(k_scatter_codes, dim3(grid_for(n)), dim3(kBlock), 0, st, stage, n, K, off, cnt, codes);
    tm.mark();  // 3
    if (part_codes_out)
      PHOBIC_HIP(hipMemcpyAsync(part_codes_out, codes, n * sizeof(ulonglong2), hipMemcpyDeviceToDevice, st));
    if (wide) {
      const size_t sort_lds = (size_t)nbpad * sizeof(uint32_t);
      if (sort_lds > max_lds_per_group())
        return fail(PHOBIC_E_CAPACITY, "B = " + std::to_string(B) + " buckets do not fit the LDS of one workgroup");
      uint32_t *wcnt, *wrank;
      PHOBIC_HIP(S.get(&wcnt, K * B));
      PHOBIC_HIP(S.get(&wrank, n));
      hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(K * B)), dim3(kBlock), 0, st, wcnt, K * B, 0u);
      PHOBIC_HIP(allow_lds(k_bucket_sort_wide, sort_lds));
      hipLaunchKernelGGL(k_bucket_sort_wide, dim3((uint32_t)K), dim3(kWideThreads), sort_lds, st, codes, off,
                         h->d_table, B, nbpad, wcnt, wrank, sortedf, blist, nbk, err);
    } else {
      const size_t sort_lds = (2 * (size_t)nbpad + std::max<uint64_t>(old_info[0], 1)) * sizeof(uint32_t);
      hipLaunchKernelGGL(k_bucket_sort, dim3((uint32_t)K), dim3(kBlock), sort_lds, st, codes, off, h->d_table, B,
                         nbpad, sortedf, blist, nbk, err + 1);
    }
    tm.mark();  // 4
    PHOBIC_HIP(hipGetLastError());
  }

  uint32_t* hinfo;  // pinned
  uint64_t* htotp;
  PHOBIC_HIP(S.host(&hinfo, 4));
  PHOBIC_HIP(S.host(&htotp, 1));
  // Minimal coarse-path builds size the search from bounds known before the data (partitions of at
  // most P + 7 sqrt(P) + 16 keys, buckets within seven standard deviations of the largest expected
  // one: exceeded about once in 10^7 builds of 10^8 keys), so the host does not wait for the
  // bucketing; a partition beyond the bounds is flagged by the search and the build repeats with
  // the exact sizes.
  const bool early = coarse_path && an == ad && !part_offsets_out && !exact_sizes;
  uint64_t max_nj, max_m, total;
  uint32_t hmaxb;
  if (early) {
    const double P = (double)prm.partition_size;
    max_nj = std::min<uint64_t>((uint64_t)std::ceil(P + 7.0 * std::sqrt(P) + 16.0), std::max<uint64_t>(n, 1));
    max_m = max_nj;
    total = n;
    hmaxb = bucket_size_bound(prm, B, max_nj);
  } else {
    PHOBIC_HIP(hipMemcpyAsync(hinfo, err, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    PHOBIC_HIP(hipMemcpyAsync(htotp, d64, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    PHOBIC_HIP(hipStreamSynchronize(st));
    if (hinfo[0] & (1u << PHOBIC_E_CAPACITY))
      return fail(PHOBIC_E_CAPACITY, wide ? "a bucket holds 65536 or more keys"
                                          : "a group of partitions exceeds the LDS of the bucket-sort workgroup");
    if (part_offsets_out) {  // hashing and partitioning only
      PHOBIC_HIP(hipMemcpyAsync(part_offsets_out, off, (K + 1) * sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
      PHOBIC_HIP(hipStreamSynchronize(st));
      return PHOBIC_OK;
    }
    max_nj = coarse_path ? hinfo[2] : old_info[0];
    max_m = coarse_path ? (an != ad ? hinfo[3] : max_nj) : old_info[1];
    total = coarse_path ? (an != ad ? *htotp : n) : old_info[2];
    hmaxb = hinfo[1];
    h->info.max_partition_keys = max_nj;
    h->info.max_bucket_keys = hmaxb;
  }
  h->info.partition_path = coarse_path ? 0u : 1u;
  if (!wide && max_m > kMaxTableSlots)
    return fail(PHOBIC_E_CAPACITY, "a partition needs " + std::to_string(max_m) + " slots; the device path holds " +
                                       std::to_string(kMaxTableSlots));

  // pilot search
  uint64_t* taken = nullptr;
  const uint64_t taken_words = (total + 63) / 64 + 1;
  if (total > n) {
    PHOBIC_HIP(S.get(&taken, taken_words));
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(taken_words)), dim3(kBlock), 0, st, taken, taken_words,
                       (uint64_t)0);
  }
  SearchArgs sa;
  sa.fp = sortedf;
  sa.off = off;
  sa.toff = toff;
  sa.blist = blist;
  sa.nbk = nbk;
  sa.pilots = pilots_pm;
  sa.err = err;
  sa.taken = taken;
  sa.K = K;
  sa.limit = limit;
  sa.B = B;
  const uint32_t mm = (uint32_t)std::max<uint64_t>(max_m, 1);
  const uint32_t mb = std::max<uint32_t>(hmaxb, 1);
  size_search_lds(sa, mm, mb, B, wide);
  if (wide && sa.wave_lds > max_lds_per_group())
    return fail(PHOBIC_E_CAPACITY, "a partition of " + std::to_string(mm) + " slots does not fit the LDS of one workgroup");
  sa.owner = nullptr;
  sa.Kbase = nullptr;
  sa.Kt = nullptr;
  sa.fail_part = nullptr;
  sa.order = nullptr;
  unsigned long long* queue;
  PHOBIC_HIP(S.get(&queue, 1));
  tm.mark();  // 5
  if (!wide && K > 1) {  // costly partitions first
    uint32_t *order, *oscr;
    PHOBIC_HIP(S.get(&order, K));
    PHOBIC_HIP(S.get(&oscr, order_scratch_words(K)));
    PHOBIC_HIP(order_partitions(sa, order, oscr, st));
  }
  PHOBIC_HIP(launch_search(sa, K, st, queue));
  tm.mark();  // 6

  // encoding: the encoders read column i (bucket i of every partition), so transpose first
  {
    const uint64_t tiles = ((K + kTile - 1) / kTile) * ((B + kTile - 1) / kTile);
    hipLaunchKernelGGL(k_transpose_u32, dim3((uint32_t)std::min<uint64_t>(tiles, 65536)), dim3(kTile, kTile / 16),
                       0, st, pilots_pm, K, (uint64_t)B, pilots);
  }
  // statistics -> host parameters, in one block so that one copy brings them back: the shifted sums
  // (B x 33), the offset residue range (2), the maxima (B u32)
  const uint64_t nstat = (uint64_t)B * 33 + 2 + (B + 1) / 2;
  uint64_t* stats;
  PHOBIC_HIP(S.get(&stats, nstat));
  uint64_t* shsum = stats;
  long long* dmm = (long long*)(stats + (uint64_t)B * 33);
  uint32_t* vmax = (uint32_t*)(stats + (uint64_t)B * 33 + 2);
  const uint64_t R = (uint64_t)(((unsigned __int128)total << 32) / K);
  hipLaunchKernelGGL(k_stats_init, dim3(grid_for(nstat)), dim3(kBlock), 0, st, stats, nstat, (uint64_t)B * 33);
  // one workgroup per (chunk, encoder) in the statistics and the packing
  const uint64_t nch = (K + kPackChunk - 1) / kPackChunk;
  uint32_t* ccnt;
  PHOBIC_HIP(S.get(&ccnt, (uint64_t)B * nch * 32));
  if (nch)
    hipLaunchKernelGGL(k_encoder_stats, dim3((uint32_t)nch, B), dim3(kBlock), 0, st, pilots, K, shsum, vmax, ccnt);
  hipLaunchKernelGGL(k_offset_stats, dim3(grid_for(K + 1, kBlock, 64)), dim3(kBlock), 0, st, toff, K, R, dmm);
  PHOBIC_HIP(hipGetLastError());
  uint64_t* hstats;  // pinned
  PHOBIC_HIP(S.host(&hstats, nstat));
  PHOBIC_HIP(hipMemcpyAsync(hstats, stats, nstat * 8, hipMemcpyDeviceToHost, st));
  PHOBIC_HIP(hipMemcpyAsync(hinfo, err, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  {  // while the device searches: take and give back a block of the likely image size (3 bits/key
     // and 40 per partition), so that the image allocation after the round trip finds mapped memory
     // in the pool instead of mapping pages on the critical path
    void* warm = nullptr;
    if (pool_alloc(&warm, (size_t)((3 * n + 40 * K) / 8) + ((size_t)B << 7) + 4096, st) == hipSuccess)
      (void)hipFreeAsync(warm, st);
    else
      (void)hipGetLastError();  // only a hint: a failure here must not surface later
  }
  PHOBIC_HIP(spin_sync(st));
  const uint64_t* hsh = hstats;
  const long long* hmm = (const long long*)(hstats + (uint64_t)B * 33);
  const uint32_t* hmax = (const uint32_t*)(hstats + (uint64_t)B * 33 + 2);
  const uint32_t herr = hinfo[0];
  if (early) {
    if (herr & (1u << PHOBIC_E_CAPACITY))
      return fail(PHOBIC_E_CAPACITY, "a group of partitions exceeds the LDS of the bucket-sort workgroup");
    if (herr & (1u << kErrResize))  // a partition or bucket beyond the bounds: size exactly
      return build_impl(in, params, st, out, nullptr, nullptr, true);
    h->info.max_partition_keys = hinfo[2];
    h->info.max_bucket_keys = hinfo[1];
  }
  if (herr & (1u << PHOBIC_E_DUPLICATE)) return fail(PHOBIC_E_DUPLICATE, "two keys of one bucket share their 64-bit fingerprint");
  if (herr & (1u << PHOBIC_E_PILOT_OVERFLOW))
    return fail(PHOBIC_E_PILOT_OVERFLOW, "a bucket needs a pilot above " + std::to_string(limit));

  const bool rice = prm.coding == PHOBIC_IC_RICE;
  const uint32_t nc = rice ? prm.n_compact : 0;  // mixed coding: encoders below nc are Compact
  std::vector<uint64_t> enc(B), ubase(B);
  uint64_t data_bits = 0, unary_bits = 0;
  for (uint32_t i = 0; i < B; i++) {
    const bool enc_rice = rice && i >= nc;
    uint32_t w = enc_rice ? rice_parameter(hsh[(size_t)i * 33], K) : bit_length(hmax[i]);
    enc[i] = (data_bits << 8) | w;
    data_bits += (uint64_t)w * K;
    if (enc_rice) {
      ubase[i] = unary_bits;
      unary_bits += hsh[(size_t)i * 33 + w] + K;
    }
  }
  if (rice && unary_bits > 0xFFFFFFFFULL)
    return fail(PHOBIC_E_CAPACITY, "the unary stream exceeds 2^32 bits");
  const long long dmin = hmm[0];
  const uint32_t woff = bit_length((uint64_t)(hmm[1] - hmm[0]));
  const uint64_t nremap = total - n;
  const uint32_t wremap = n > 1 ? bit_length(n - 1) : 0;
  const std::vector<uint64_t> hdr = make_header(n, K, B, prm, total, dmin, woff, data_bits, unary_bits, R);
  const uint64_t nwords = hdr[kHWords];

  PHOBIC_HIP(pool_alloc((void**)&h->d_image, nwords * sizeof(uint64_t), st));
  h->nwords = nwords;
  h->header = hdr;
  uint64_t* img = h->d_image;
  // header, encoder words and unary bases go over in one copy; the image is zeroed and its header
  // and encoder words set by one kernel
  std::vector<uint64_t> hw(hdr.begin(), hdr.begin() + kHeaderWords);
  hw.insert(hw.end(), enc.begin(), enc.end());
  if (rice) hw.insert(hw.end(), ubase.begin(), ubase.end());
  uint64_t* dhw;
  PHOBIC_HIP(S.get(&dhw, hw.size()));
  PHOBIC_HIP(S.upload(dhw, hw.data(), hw.size()));
  hipLaunchKernelGGL(k_image_init, dim3(grid_for(nwords)), dim3(kBlock), 0, st, img, nwords, dhw,
                     (uint32_t)kHeaderWords, hdr[kHSecEnc], B);
  uint64_t* carries = nullptr;
  if (rice && nch) {
    PHOBIC_HIP(S.get(&carries, (uint64_t)B * nch));
    if (B > nc)
      hipLaunchKernelGGL(k_chunk_carry, dim3(B - nc), dim3(kBlock), 0, st, ccnt, K, nch, dhw + kHeaderWords,
                         dhw + kHeaderWords + B, carries, nc);
  }
  if (woff)
    hipLaunchKernelGGL(k_pack_offsets, dim3(grid_for(K + 1)), dim3(kBlock), 0, st, toff, K, R, dmin, woff,
                       img + hdr[kHSecOff]);
  if (nch)
    hipLaunchKernelGGL(k_pack_values, dim3((uint32_t)nch, B), dim3(kPackThreads), 0, st, pilots, K,
                       img + hdr[kHSecEnc], carries, (uint32_t)rice, nc, img + hdr[kHSecData],
                       img + hdr[kHSecUnary], img + hdr[kHSecSel]);
  const uint64_t nvals = K * (B - nc);  // ones of the unary stream: the values of the Rice encoders
  if (rice && nvals)
    hipLaunchKernelGGL(k_sel_fill, dim3(grid_for((nvals + kSelBlock - 1) / kSelBlock)), dim3(kBlock), 0, st,
                       img + hdr[kHSecUnary], img + hdr[kHSecSel], (nvals + kSelBlock - 1) / kSelBlock, nvals);
  PHOBIC_HIP(hipGetLastError());
  if (nremap && wremap) {
    uint32_t *fc, *oc, *freeslot;
    PHOBIC_HIP(S.get(&fc, taken_words));
    PHOBIC_HIP(S.get(&oc, taken_words));
    PHOBIC_HIP(S.get(&freeslot, nremap));
    hipLaunchKernelGGL(k_remap_count, dim3(grid_for(taken_words)), dim3(kBlock), 0, st, taken, taken_words, n, total,
                       fc, oc);
    const uint64_t nsb = (taken_words + kScanBlock - 1) / kScanBlock;
    uint64_t* bsums;
    PHOBIC_HIP(S.get(&bsums, 2 * nsb));
    hipLaunchKernelGGL(k_pair_block_sums, dim3((uint32_t)nsb), dim3(kScanThreads), 0, st, fc, oc, taken_words, bsums);
    hipLaunchKernelGGL(k_pair_scan_blocks, dim3(1), dim3(kScanThreads), 0, st, bsums, nsb);
    hipLaunchKernelGGL(k_pair_apply, dim3((uint32_t)nsb), dim3(kScanThreads), 0, st, fc, oc, taken_words, bsums);
    hipLaunchKernelGGL(k_remap_free, dim3(grid_for(taken_words)), dim3(kBlock), 0, st, taken, taken_words, n, fc,
                       freeslot);
    hipLaunchKernelGGL(k_remap_fill, dim3(grid_for(nremap)), dim3(kBlock), 0, st, taken, n, total, oc, freeslot,
                       wremap, img + hdr[kHSecRemap]);
    PHOBIC_HIP(hipGetLastError());
  }
  tm.mark();  // 7
  PHOBIC_HIP(spin_sync(st));
  auto t_host1 = std::chrono::steady_clock::now();

  h->info.hash_count_ms = tm.ms(0, 1);
  h->info.scan_ms = tm.ms(1, 2);
  h->info.scatter_ms = tm.ms(2, 3);
  h->info.bucket_sort_ms = tm.ms(3, 4);
  h->info.search_ms = tm.ms(5, 6);
  h->info.encode_ms = tm.ms(6, 7);
  h->info.total_ms = std::chrono::duration<double, std::milli>(t_host1 - t_host0).count();
  fill_query_args(h);
  *out = h;
  h = nullptr;  // ownership moves to the caller
  return PHOBIC_OK;
}


// ---------------------------------------------------------------------------------------------
// Batched builds.  The partitions of all MPHFs form one global index space (MPHF t owns
// [Kbase_t, Kbase_t + K_t)) and their keys one global key space (MPHF t owns
// [nbase_t, nbase_t + n_t)).  Every per-partition step is the plain build's; only the mapping
// from a key to its global partition and from a partition to its MPHF is new.
// ---------------------------------------------------------------------------------------------
struct BatchDesc {
  const uint64_t* keys;
  uint64_t n, K, Kbase, nbase, R;  // R = floor(n 2^32 / K), the offset expectation step
};

// the last MPHF t in [lo, hi) with nbase_t <= gi (empty MPHFs share nbase with their successor)
__device__ __forceinline__ uint32_t batch_owner(const BatchDesc* __restrict__ d, uint32_t lo, uint32_t hi,
                                                uint64_t gi) {
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (d[mid].nbase <= gi) lo = mid; else hi = mid;
  }
  return lo;
}

template <bool kScatter>
__global__ __launch_bounds__(kCoarseThreads) void k_batch_coarse(const BatchDesc* __restrict__ d, uint32_t t0,
                                                                 uint32_t t1, uint64_t nb0, uint64_t nchunk,
                                                                 uint64_t per, uint64_t seed, uint64_t Jc0,
                                                                 uint32_t gshift, uint32_t C,
                                                                 uint32_t* __restrict__ ccnt, uint32_t* __restrict__ hrow,
                                                                 uint32_t* __restrict__ cur,
                                                                 ulonglong2* __restrict__ codes) {
  extern __shared__ __align__(16) uint32_t hist[];
  const uint32_t tid = threadIdx.x;
  if (kScatter) {
    for (uint32_t x = tid; x < C; x += kCoarseThreads) {
      const uint32_t v = hrow[(uint64_t)blockIdx.x * C + x];
      hist[x] = v ? atomicAdd(&cur[x], v) : 0u;
    }
  } else {
    for (uint32_t x = tid; x < C; x += kCoarseThreads) hist[x] = 0;
  }
  __syncthreads();
  const uint64_t a = (uint64_t)blockIdx.x * per, b = min(nchunk, a + per);
  // the thread's keys only move forward, and so does their MPHF t: its fields stay in registers and
  // are reloaded only where the next MPHF starts (empty MPHFs share nbase with their successor), so
  // that a key's load does not wait on loads of its descriptor
  uint32_t t = a + tid < b ? batch_owner(d, t0, t1, nb0 + a + tid) : t0;
  uint64_t tnb = d[t].nbase, tK = d[t].K, tKb = d[t].Kbase;
  uint64_t tnext = t + 1 < t1 ? d[t + 1].nbase : ~0ULL;
  const uint64_t* tkeys = d[t].keys;
  const uint64_t gmask = (1ULL << gshift) - 1;
  // four keys per thread and round, loaded before any is hashed, so that the loads are in flight
  // together
  constexpr int kU = 4;
  for (uint64_t i0 = a + tid; i0 < b; i0 += (uint64_t)kU * kCoarseThreads) {
    uint64_t key[kU], kK[kU], kKb[kU];
#pragma unroll
    for (int u = 0; u < kU; u++) {
      const uint64_t gi = nb0 + min(i0 + (uint64_t)u * kCoarseThreads, b - 1);
      while (gi >= tnext) {
        t++;
        tnb = tnext;
        tK = d[t].K;
        tKb = d[t].Kbase;
        tkeys = d[t].keys;
        tnext = t + 1 < t1 ? d[t + 1].nbase : ~0ULL;
      }
      key[u] = tkeys[gi - tnb];
      kK[u] = tK;
      kKb[u] = tKb;
    }
#pragma unroll
    for (int u = 0; u < kU; u++) {
      if (i0 + (uint64_t)u * kCoarseThreads >= b) break;
      const uint64_t J = kKb[u] + __umul64hi(mix_a(key[u] ^ seed), kK[u]);
      const uint32_t bin = (uint32_t)((J - Jc0) >> gshift);
      if (kScatter) {
        uint64_t hi, lo;
        hash_key_u64(key[u], seed, hi, lo);
        codes[atomicAdd(&hist[bin], 1u)] = make_ulonglong2(fingerprint(hi, lo), (lo & ~7ULL) | ((J - Jc0) & gmask));
      } else {
        atomicAdd(&hist[bin], 1u);
      }
    }
  }
  if (!kScatter) {
    __syncthreads();
    for (uint32_t x = tid; x < C; x += kCoarseThreads) {
      const uint32_t v = hist[x];
      hrow[(uint64_t)blockIdx.x * C + x] = v;
      if (v) atomicAdd(&ccnt[x], v);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_batch_owner(const BatchDesc* __restrict__ d, uint32_t count, uint64_t Ktot,
                                                        uint32_t* __restrict__ owner) {
  for (uint64_t J = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; J < Ktot; J += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t lo = 0, hi = count;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (d[mid].Kbase <= J) lo = mid; else hi = mid;
    }
    owner[J] = lo;
  }
}

// Statistics of every (MPHF t, encoder i) item: 16 lanes per item, 16 items per workgroup (most
// items hold a few dozen values, so a wavefront per item would spend its time reducing).
constexpr uint32_t kItemLanes = 16, kItemsPerGroup = 256 / kItemLanes;
__device__ __forceinline__ uint64_t item_sum_u64(uint64_t v) {
#pragma unroll
  for (int o = 1; o < (int)kItemLanes; o <<= 1) v += __shfl_xor(v, o, kItemLanes);
  return v;
}

// sum and maximum of the item's values
__global__ __launch_bounds__(256) void k_batch_stats(const uint32_t* __restrict__ pilots,
                                                     const BatchDesc* __restrict__ d, uint32_t count, uint32_t B,
                                                     uint64_t* __restrict__ sum, uint32_t* __restrict__ mx) {
  const uint64_t item = (uint64_t)blockIdx.x * kItemsPerGroup + threadIdx.x / kItemLanes;
  const uint32_t q = threadIdx.x % kItemLanes;
  const bool ok = item < (uint64_t)count * B;
  const uint32_t t = ok ? (uint32_t)(item / B) : 0u, i = ok ? (uint32_t)(item % B) : 0u;
  const uint64_t K = ok ? d[t].K : 0;
  const uint32_t* col = pilots + (uint64_t)B * (ok ? d[t].Kbase : 0) + (uint64_t)i * K;
  uint64_t s = 0;
  uint32_t m = 0;
  for (uint64_t j = q; j < K; j += kItemLanes) {
    const uint32_t v = col[j];
    s += v;
    m = max(m, v);
  }
  s = item_sum_u64(s);
#pragma unroll
  for (int o = 1; o < (int)kItemLanes; o <<= 1) m = max(m, (uint32_t)__shfl_xor(m, o, kItemLanes));
  if (ok && q == 0) {
    sum[item] = s;
    mx[item] = m;
  }
}

// bits of the item's unary stream: sum (v >> w) + K_t
__global__ __launch_bounds__(256) void k_batch_unary(const uint32_t* __restrict__ pilots,
                                                     const BatchDesc* __restrict__ d, uint32_t count, uint32_t B,
                                                     const uint8_t* __restrict__ width, uint64_t* __restrict__ ubits) {
  const uint64_t item = (uint64_t)blockIdx.x * kItemsPerGroup + threadIdx.x / kItemLanes;
  const uint32_t q = threadIdx.x % kItemLanes;
  const bool ok = item < (uint64_t)count * B;
  const uint32_t t = ok ? (uint32_t)(item / B) : 0u, i = ok ? (uint32_t)(item % B) : 0u;
  const uint64_t K = ok ? d[t].K : 0;
  const uint32_t w = ok ? width[item] : 0u;
  const uint32_t* col = pilots + (uint64_t)B * (ok ? d[t].Kbase : 0) + (uint64_t)i * K;
  uint64_t s = 0;
  for (uint64_t j = q; j < K; j += kItemLanes) s += (uint64_t)col[j] >> w;
  s = item_sum_u64(s);
  if (ok && q == 0) ubits[item] = s + K;
}

// One wavefront per MPHF: minimum and maximum offset residue.
__global__ __launch_bounds__(256) void k_batch_offstats(const uint64_t* __restrict__ off,
                                                        const BatchDesc* __restrict__ d, uint32_t count,
                                                        long long* __restrict__ mm) {
  const uint32_t t = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (t >= count) return;
  const BatchDesc e = d[t];
  long long lmin = LLONG_MAX, lmax = LLONG_MIN;
  for (uint64_t j = lane; j <= e.K; j += 64) {
    const long long v = (long long)((off[e.Kbase + j] - e.nbase) - expected_offset(j, e.R));
    lmin = min(lmin, v);
    lmax = max(lmax, v);
  }
  for (int o = 32; o > 0; o >>= 1) {
    lmin = min(lmin, (long long)__shfl_xor(lmin, o));
    lmax = max(lmax, (long long)__shfl_xor(lmax, o));
  }
  if (lane == 0) {
    mm[2 * t] = lmin;
    mm[2 * t + 1] = lmax;
  }
}

// Encoder widths of every (MPHF t, encoder i): Kiely's parameter of the mean (Rice encoders) from
// the thresholds the host found with the same formula, else the bit length of the maximum.
__global__ __launch_bounds__(kBlock) void k_batch_widths(const BatchDesc* __restrict__ d, uint32_t count, uint32_t B,
                                                         const uint64_t* __restrict__ sum,
                                                         const uint32_t* __restrict__ mx, uint32_t rice, uint32_t ncomp,
                                                         RiceThresholds th, uint8_t* __restrict__ width) {
  for (uint64_t it = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; it < (uint64_t)count * B;
       it += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t t = (uint32_t)(it / B), i = (uint32_t)(it % B);
    const uint32_t v = mx[it];
    width[it] = (uint8_t)(rice && i >= ncomp ? rice_from_thresholds(sum[it], d[t].K, th) : (v ? 32 - __clz(v) : 0));
  }
}

// Everything an image's packing needs that depends on the whole MPHF, one thread per MPHF: encoder
// words (data bit base << 8 | width), unary bases, the header, and the image's size in words.
struct BatchPlan {
  uint64_t lambda_bits, alpha_word, coding_word, seed;
  uint32_t P, ncomp;
};

// One wavefront per MPHF (four per workgroup): the encoders' bit bases are prefix sums over the
// encoders in order, taken 64 encoders at a time with a wavefront scan.
constexpr uint32_t kPlanWaves = 4;
__global__ __launch_bounds__(64 * kPlanWaves) void k_batch_plan(const BatchDesc* __restrict__ d, uint32_t count,
                                                                uint32_t B, const uint8_t* __restrict__ width,
                                                                const uint64_t* __restrict__ ubits,
                                                                const long long* __restrict__ mm, BatchPlan pl,
                                                                uint64_t* __restrict__ encw,
                                                                uint64_t* __restrict__ ubase,
                                                                uint64_t* __restrict__ hdrs,
                                                                uint64_t* __restrict__ words,
                                                                uint32_t* __restrict__ err) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t t = blockIdx.x * kPlanWaves + (threadIdx.x >> 6);
  if (t >= count) return;  // whole wavefronts leave together
  const BatchDesc e = d[t];
  const bool rice = (pl.coding_word & 0xFF) == PHOBIC_IC_RICE;
  uint64_t data_bits = 0, unary_bits = 0;  // totals of the encoders before the current 64
  for (uint32_t i0 = 0; i0 < B; i0 += 64) {
    const uint32_t i = i0 + lane;
    const uint64_t it = (uint64_t)t * B + i;
    const uint32_t w = i < B ? width[it] : 0u;
    uint64_t db = (uint64_t)w * e.K;
    uint64_t ub = i < B && rice && i >= pl.ncomp ? ubits[it] : 0;  // Compact encoders have no unary part
    // inclusive wavefront scans of both
    uint64_t sdb = db, sub = ub;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint64_t a = __shfl_up(sdb, o), b = __shfl_up(sub, o);
      if (lane >= (uint32_t)o) {
        sdb += a;
        sub += b;
      }
    }
    if (i < B) {
      encw[it] = ((data_bits + sdb - db) << 8) | w;
      ubase[it] = unary_bits + sub - ub;
    }
    data_bits += __shfl(sdb, 63);
    unary_bits += __shfl(sub, 63);
  }
  if (lane != 0) return;
  if (rice && unary_bits > 0xFFFFFFFFULL) atomicOr(&err[0], 1u << PHOBIC_E_CAPACITY);
  const long long dmin = mm[2 * t], dmax = mm[2 * t + 1];
  const uint64_t span = (uint64_t)(dmax - dmin);
  const uint32_t woff = span ? 64 - __clzll(span) : 0;
  uint64_t* h = hdrs + (uint64_t)t * kHeaderWords;
  uint64_t hv[kHeaderWords];
  fill_header(hv, e.n, e.K, B, pl.P, pl.lambda_bits, pl.alpha_word, pl.coding_word, pl.seed, e.n, dmin, woff,
              data_bits, unary_bits, e.R, pl.ncomp);
  for (uint32_t x = 0; x < kHeaderWords; x++) h[x] = hv[x];
  words[t] = hv[kHWords];
}

// One workgroup per MPHF: header and encoder words into its image.
__global__ __launch_bounds__(256) void k_batch_heads(const uint64_t* __restrict__ hdrs, const uint64_t* __restrict__ encw,
                                                     const uint64_t* __restrict__ ibase, uint32_t B,
                                                     uint64_t* __restrict__ buf) {
  const uint32_t t = blockIdx.x;
  const uint64_t* h = hdrs + (uint64_t)t * kHeaderWords;
  uint64_t* img = buf + ibase[t];
  for (uint32_t x = threadIdx.x; x < kHeaderWords; x += blockDim.x) img[x] = h[x];
  for (uint32_t x = threadIdx.x; x < B; x += blockDim.x) img[h[kHSecEnc] + x] = encw[(uint64_t)t * B + x];
}

// One wavefront per MPHF: offset residues into the OFF section.
__global__ __launch_bounds__(256) void k_batch_pack_off(const uint64_t* __restrict__ off, const BatchDesc* __restrict__ d,
                                                        uint32_t count, const uint64_t* __restrict__ hdrs,
                                                        const uint64_t* __restrict__ ibase, uint64_t* __restrict__ buf) {
  const uint32_t t = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (t >= count) return;
  const BatchDesc e = d[t];
  const uint64_t* h = hdrs + (uint64_t)t * kHeaderWords;
  const long long dmin = (long long)h[kHDmin];
  const uint32_t woff = (uint32_t)h[kHWoff];
  uint64_t* sec = buf + ibase[t] + h[kHSecOff];
  for (uint64_t j = lane; j <= e.K; j += 64) {
    const uint64_t u = (uint64_t)((long long)((off[e.Kbase + j] - e.nbase) - expected_offset(j, e.R)) - dmin);
    put_bits_atomic(sec, j * woff, u, woff);
  }
}

// One wavefront per (t, i): values (Compact) or low bits and unary stream with select samples (Rice).
// One wavefront per (MPHF t, encoder i), 64 values at a time: the chunk's low bits (64 fields of at
// most 32 bits) and, when they fit, its unary bits are assembled in the wavefront's LDS and written
// as whole words, with an atomic OR only on the two end words a neighbouring chunk or item may share
// (the same scheme as k_pack_values).
constexpr uint32_t kBatchDataWords = 34;   // 64 x 32 bits + two partial words
constexpr uint32_t kBatchUnaryWords = 64;  // unary runs of up to 64 x 64 - 63 bits are staged

__device__ __forceinline__ void wave_flush_words(const uint64_t* lbuf, uint64_t* __restrict__ dst, uint64_t first,
                                                 uint32_t last, uint32_t lane) {
  for (uint32_t x = lane; x <= last; x += 64) {
    const uint64_t v = lbuf[x];
    if (x == 0 || x == last) {
      if (v) atomicOr((unsigned long long*)&dst[first + x], (unsigned long long)v);
    } else {
      dst[first + x] = v;
    }
  }
}

__global__ __launch_bounds__(256) void k_batch_pack_vals(const uint32_t* __restrict__ pilots,
                                                         const BatchDesc* __restrict__ d, uint32_t count, uint32_t B,
                                                         const uint64_t* __restrict__ hdrs,
                                                         const uint64_t* __restrict__ encw,
                                                         const uint64_t* __restrict__ ubase,
                                                         const uint64_t* __restrict__ ibase, uint64_t* __restrict__ buf) {
  __shared__ uint64_t lds_d[4][kBatchDataWords];
  __shared__ uint64_t lds_u[4][kBatchUnaryWords];
  const uint32_t wv = threadIdx.x >> 6;
  uint64_t* dbuf = lds_d[wv];
  uint64_t* ubuf = lds_u[wv];
  const uint64_t item = (uint64_t)blockIdx.x * 4 + wv;
  const uint32_t lane = threadIdx.x & 63;
  if (item >= (uint64_t)count * B) return;
  const uint32_t t = (uint32_t)(item / B), i = (uint32_t)(item % B);
  const uint64_t K = d[t].K;
  const uint64_t* h = hdrs + (uint64_t)t * kHeaderWords;
  uint64_t* img = buf + ibase[t];
  uint64_t* data = img + h[kHSecData];
  uint64_t* unary = img + h[kHSecUnary];
  const uint32_t nc = (uint32_t)h[kHNcompact];  // mixed coding: encoders below nc are Compact
  const bool rice = (h[kHCoding] & 0xFF) == PHOBIC_IC_RICE && i >= nc;
  const uint64_t e = encw[item];
  const uint32_t w = (uint32_t)(e & 0xFF);
  const uint64_t base = e >> 8;
  const uint32_t* col = pilots + (uint64_t)B * d[t].Kbase + (uint64_t)i * K;
  uint64_t carry = rice ? ubase[item] : 0;
  for (uint64_t j0 = 0; j0 < K; j0 += 64) {
    const uint64_t j = j0 + lane;
    const bool in = j < K;
    const uint64_t v = in ? col[j] : 0;
    if (lane < kBatchDataWords) dbuf[lane] = 0;
    ubuf[lane] = 0;
    const uint64_t jend = min(K, j0 + 64);
    uint64_t incl = 0, tot = 0;
    if (rice) {
      incl = in ? (v >> w) + 1 : 0;
      for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(incl, o);
        if (lane >= (uint32_t)o) incl += y;
      }
      tot = __shfl(incl, 63);
    }
    const uint64_t d_first = (base + j0 * w) >> 6, u_first = carry >> 6;
    const bool u_lds = tot == 0 || ((carry + tot - 1) >> 6) - u_first < kBatchUnaryWords;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (in && w) {
      const uint64_t rel = base + j * w - d_first * 64;
      const uint32_t idx = (uint32_t)(rel >> 6), sh = (uint32_t)(rel & 63);
      const uint64_t f = v & ((1ULL << w) - 1);
      atomicOr((unsigned long long*)&dbuf[idx], (unsigned long long)(f << sh));
      if (sh + w > 64) atomicOr((unsigned long long*)&dbuf[idx + 1], (unsigned long long)(f >> (64 - sh)));
    }
    if (rice && in) {
      const uint64_t pos = carry + incl - 1;  // this value's one
      if (u_lds)
        atomicOr((unsigned long long*)&ubuf[(pos >> 6) - u_first], 1ULL << (pos & 63));
      else
        atomicOr((unsigned long long*)&unary[pos >> 6], 1ULL << (pos & 63));
      const uint64_t tg = (uint64_t)(i - nc) * K + j;
      if ((tg & (kSelBlock - 1)) == 0) img[h[kHSecSel] + tg / kSelBlock] = pos;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (w) wave_flush_words(dbuf, data, d_first, (uint32_t)(((base + jend * w - 1) >> 6) - d_first), lane);
    if (rice && u_lds && tot) wave_flush_words(ubuf, unary, u_first, (uint32_t)(((carry + tot - 1) >> 6) - u_first), lane);
    carry += tot;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// Sub-sample distances of the select entries of every MPHF of a batch, one workgroup per MPHF.
__global__ __launch_bounds__(256) void k_batch_sel_fill(const BatchDesc* __restrict__ d, uint32_t B,
                                                        const uint64_t* __restrict__ hdrs,
                                                        const uint64_t* __restrict__ ibase, uint64_t* __restrict__ buf) {
  const uint32_t t = blockIdx.x;
  const uint64_t* h = hdrs + (uint64_t)t * kHeaderWords;
  uint64_t* img = buf + ibase[t];
  const uint64_t nvals = d[t].K * (B - h[kHNcompact]), nsel = (nvals + kSelBlock - 1) / kSelBlock;
  for (uint64_t s = threadIdx.x; s < nsel; s += blockDim.x) sel_fill_entry(img + h[kHSecUnary], img + h[kHSecSel], s, nvals);
}

phobic_status build_batch_impl(const uint64_t* const* keys, const uint64_t* counts, uint32_t count,
                               const phobic_params* params, hipStream_t st, phobic_mphf** outs) {
  uint32_t B = 0;
  phobic_status vs = validate_params(params, &B);
  if (vs != PHOBIC_OK) return vs;
  const phobic_params& prm = *params;
  if (prm.alpha_num != prm.alpha_den) return fail(PHOBIC_E_INVALID, "batched builds need alpha = 1");
  if (B > kMaxBuckets) return fail(PHOBIC_E_CAPACITY, "B exceeds the device limit");
  configure_pool_once();
  const uint32_t nbpad = next_pow2(B);
  int gshift = -1;
  uint32_t seg_cap = 0;
  for (int gs = 3; gs >= 0; gs--) {
    const double gp = (double)(1u << gs) * prm.partition_size;
    const int64_t cap = ((int64_t)kSegLdsBytes - 8 * (int64_t)(1u << gs) * nbpad) / 4;
    if (cap > 0 && gp + 8.0 * std::sqrt(gp) + 64.0 <= (double)cap) {
      gshift = gs;
      seg_cap = (uint32_t)cap;
      break;
    }
  }
  if (gshift < 0) return fail(PHOBIC_E_CAPACITY, "partition_size too large for batched builds");
  const uint64_t G = 1ULL << gshift;
  uint64_t chunk_parts = (uint64_t)kMaxCoarse * G;
  // PHOBIC_BATCH_CHUNK_PARTS lowers the partitions handled per chunk (tests use it to exercise
  // several chunks with small batches); it never changes a result.
  if (const char* env = std::getenv("PHOBIC_BATCH_CHUNK_PARTS")) {
    const uint64_t v = std::strtoull(env, nullptr, 10);
    if (v >= 1) chunk_parts = std::min<uint64_t>(chunk_parts, v);
  }
  const uint64_t limit = prm.pilot_limit ? prm.pilot_limit : 0xFFFFFFFFULL;

  // host descriptors and chunks of whole MPHFs
  std::vector<BatchDesc> desc(count);
  std::vector<uint64_t> hKbase(count), hKt(count);
  uint64_t Ktot = 0, Ntot = 0;
  for (uint32_t t = 0; t < count; t++) {
    const uint64_t n = counts[t];
    if (n && !keys[t]) return fail(PHOBIC_E_INVALID, "MPHF " + std::to_string(t) + ": null key pointer");
    const uint64_t K = num_partitions(n, prm.partition_size);
    if (K > chunk_parts || n >= (1ULL << 31))
      return fail(PHOBIC_E_CAPACITY, "MPHF " + std::to_string(t) + " is too large for a batch; build it alone");
    desc[t] = BatchDesc{keys[t], n, K, Ktot, Ntot, (uint64_t)(((unsigned __int128)n << 32) / K)};
    hKbase[t] = Ktot;
    hKt[t] = K;
    Ktot += K;
    Ntot += n;
  }
  struct Chunk { uint32_t t0, t1; };
  std::vector<Chunk> chunks;
  for (uint32_t t = 0; t < count;) {
    uint32_t u = t;
    uint64_t kc = 0, nc = 0;
    while (u < count && kc + desc[u].K <= chunk_parts && nc + desc[u].n < (1ULL << 31)) {
      kc += desc[u].K;
      nc += desc[u].n;
      u++;
    }
    chunks.push_back({t, u});
    t = u;
  }
  uint64_t max_chunk_keys = 0;
  for (auto& c : chunks)
    max_chunk_keys = std::max<uint64_t>(max_chunk_keys,
                                        desc[c.t1 - 1].nbase + desc[c.t1 - 1].n - desc[c.t0].nbase);

  int dev = 0;
  PHOBIC_HIP(hipGetDevice(&dev));
  phobic_mphf tbl;  // borrows the cached bucket-function table
  tbl.device = dev;
  tbl.prm = prm;
  {
    phobic_status ts = upload_table(&tbl, st);
    if (ts != PHOBIC_OK) return ts;
  }

  Scratch S(st);
  Timer tm(st);
  auto t_host0 = std::chrono::steady_clock::now();
  BatchDesc* d_desc;
  uint64_t *fp, *off, *d_Kbase, *d_Kt, *cbase;
  uint32_t *blist, *nbk, *pilots, *err, *owner, *ccnt, *hrow, *cur;
  ulonglong2* codes;
  unsigned long long* queue;
  const uint32_t ngrp_max = kCoarseGroups;
  PHOBIC_HIP(S.get(&d_desc, count));
  PHOBIC_HIP(S.get(&fp, Ntot));
  PHOBIC_HIP(S.get(&off, Ktot + 1));
  PHOBIC_HIP(S.get(&d_Kbase, count));
  PHOBIC_HIP(S.get(&d_Kt, count));
  PHOBIC_HIP(S.get(&cbase, kMaxCoarse + 1));
  PHOBIC_HIP(S.get(&blist, Ktot * B));
  PHOBIC_HIP(S.get(&nbk, Ktot));
  PHOBIC_HIP(S.get(&pilots, Ktot * B));
  PHOBIC_HIP(S.get(&err, 6));
  PHOBIC_HIP(S.get(&owner, Ktot));
  PHOBIC_HIP(S.get(&ccnt, kMaxCoarse));
  PHOBIC_HIP(S.get(&hrow, (uint64_t)ngrp_max * kMaxCoarse));
  PHOBIC_HIP(S.get(&cur, kMaxCoarse));
  PHOBIC_HIP(S.get(&codes, max_chunk_keys));
  PHOBIC_HIP(S.get(&queue, 1));
  PHOBIC_HIP(hipMemcpyAsync(d_desc, desc.data(), count * sizeof(BatchDesc), hipMemcpyHostToDevice, st));
  PHOBIC_HIP(hipMemcpyAsync(d_Kbase, hKbase.data(), count * 8, hipMemcpyHostToDevice, st));
  PHOBIC_HIP(hipMemcpyAsync(d_Kt, hKt.data(), count * 8, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(Ktot * B)), dim3(kBlock), 0, st, pilots, Ktot * B, 0u);
  // err[0] error bits, [1] max bucket, [2] max n_j, [3] max m_j; err[4..5] the lowest failing partition
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, err, (uint64_t)4, 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, err + 4, (uint64_t)2, 0xFFFFFFFFu);

  // hash, partition, bucket and order, chunk by chunk
  tm.mark();  // 0
  for (const Chunk& c : chunks) {
    const uint64_t Jc0 = desc[c.t0].Kbase, Jc1 = desc[c.t1 - 1].Kbase + desc[c.t1 - 1].K;
    const uint64_t nb0 = desc[c.t0].nbase, nchunk = desc[c.t1 - 1].nbase + desc[c.t1 - 1].n - nb0;
    const uint64_t C = (Jc1 - Jc0 + G - 1) >> gshift;
    const uint32_t ngrp = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(ngrp_max, (nchunk + 4095) / 4096));
    const uint64_t per = (nchunk + ngrp - 1) / ngrp;
    const size_t hist_lds = C * sizeof(uint32_t);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(C)), dim3(kBlock), 0, st, ccnt, C, 0u);
    hipLaunchKernelGGL(k_batch_coarse<false>, dim3(ngrp), dim3(kCoarseThreads), hist_lds, st, d_desc, c.t0, c.t1, nb0,
                       nchunk, per, prm.hash_seed, Jc0, (uint32_t)gshift, (uint32_t)C, ccnt, hrow, cur, codes);
    hipLaunchKernelGGL(k_coarse_scan, dim3(1), dim3(1024), 0, st, ccnt, (uint32_t)C, cbase, cur);
    hipLaunchKernelGGL(k_batch_coarse<true>, dim3(ngrp), dim3(kCoarseThreads), hist_lds, st, d_desc, c.t0, c.t1, nb0,
                       nchunk, per, prm.hash_seed, Jc0, (uint32_t)gshift, (uint32_t)C, ccnt, hrow, cur, codes);
    hipLaunchKernelGGL(k_segment_sort<kInRecords>, dim3((uint32_t)C), dim3(kSegThreads), kSegLdsBytes, st,
                       (const void*)codes, prm.hash_seed, cbase, tbl.d_table, B, nbpad, (uint32_t)gshift, (uint64_t)0,
                       Jc0, Jc1, nb0, seg_cap, fp, blist, nbk, off, err, (ulonglong2*)nullptr);
    PHOBIC_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_batch_owner, dim3(grid_for(Ktot)), dim3(kBlock), 0, st, d_desc, count, Ktot, owner);
  tm.mark();  // 1
  uint32_t hinfo[4];
  PHOBIC_HIP(hipMemcpyAsync(hinfo, err, sizeof(hinfo), hipMemcpyDeviceToHost, st));
  PHOBIC_HIP(spin_sync(st));
  if (hinfo[0] & (1u << PHOBIC_E_CAPACITY))
    return fail(PHOBIC_E_CAPACITY, "a group of partitions exceeds the LDS of the bucket-sort workgroup");
  if (hinfo[2] > kMaxTableSlots)
    return fail(PHOBIC_E_CAPACITY, "a partition holds " + std::to_string(hinfo[2]) + " keys; the device path holds " +
                                       std::to_string(kMaxTableSlots));

  // one pilot search over every (MPHF, partition)
  SearchArgs sa;
  sa.fp = fp;
  sa.off = off;
  sa.toff = off;
  sa.blist = blist;
  sa.nbk = nbk;
  sa.pilots = pilots;
  sa.err = err;
  sa.taken = nullptr;
  sa.K = Ktot;
  sa.limit = limit;
  sa.B = B;
  const uint32_t mm = std::max<uint32_t>(hinfo[2], 1), mb = std::max<uint32_t>(hinfo[1], 1);
  size_search_lds(sa, mm, mb, B, false);
  sa.owner = owner;
  sa.Kbase = d_Kbase;
  sa.Kt = d_Kt;
  sa.fail_part = (unsigned long long*)(err + 4);
  sa.order = nullptr;
  tm.mark();  // 2
  if (Ktot > 1) {  // costly partitions of all MPHFs first
    uint32_t *order, *oscr;
    PHOBIC_HIP(S.get(&order, Ktot));
    PHOBIC_HIP(S.get(&oscr, order_scratch_words(Ktot)));
    PHOBIC_HIP(order_partitions(sa, order, oscr, st));
  }
  PHOBIC_HIP(launch_search(sa, Ktot, st, queue));
  tm.mark();  // 3

  // encoding: statistics, then every encoder's parameter and every MPHF's header planned on the
  // device; the host learns only the image sizes (one round trip) to allocate them
  const uint64_t items = (uint64_t)count * B;
  const bool rice = prm.coding == PHOBIC_IC_RICE;
  const uint32_t ncomp = rice ? prm.n_compact : 0;  // mixed coding: encoders below it are Compact
  uint64_t *sum, *dub, *dh, *de, *du, *dib, *dwords;
  uint32_t* mx;
  uint8_t* dw;
  long long* dmm;
  PHOBIC_HIP(S.get(&sum, items));
  PHOBIC_HIP(S.get(&mx, items));
  PHOBIC_HIP(S.get(&dmm, 2 * (uint64_t)count));
  PHOBIC_HIP(S.get(&dw, items));
  PHOBIC_HIP(S.get(&dub, items));
  PHOBIC_HIP(S.get(&dh, (uint64_t)count * kHeaderWords));
  PHOBIC_HIP(S.get(&de, items));
  PHOBIC_HIP(S.get(&du, items));
  PHOBIC_HIP(S.get(&dib, count));
  PHOBIC_HIP(S.get(&dwords, count));
  const uint32_t item_groups = (uint32_t)((items + 3) / 4), mphf_groups = (count + 3) / 4;
  const uint32_t stat_groups = (uint32_t)((items + kItemsPerGroup - 1) / kItemsPerGroup);
  hipLaunchKernelGGL(k_batch_stats, dim3(stat_groups), dim3(256), 0, st, pilots, d_desc, count, B, sum, mx);
  hipLaunchKernelGGL(k_batch_offstats, dim3(mphf_groups), dim3(256), 0, st, off, d_desc, count, dmm);
  hipLaunchKernelGGL(k_batch_widths, dim3(grid_for(items)), dim3(kBlock), 0, st, d_desc, count, B, sum, mx,
                     (uint32_t)rice, ncomp, rice_thresholds(), dw);
  if (rice)
    hipLaunchKernelGGL(k_batch_unary, dim3(stat_groups), dim3(256), 0, st, pilots, d_desc, count, B, dw, dub);
  BatchPlan plan;
  std::memcpy(&plan.lambda_bits, &prm.lambda, 8);
  plan.alpha_word = (uint64_t)prm.alpha_num | ((uint64_t)prm.alpha_den << 32);
  plan.coding_word = prm.coding | ((uint64_t)prm.bucket_function << 8);
  plan.seed = prm.hash_seed;
  plan.P = prm.partition_size;
  plan.ncomp = ncomp;
  hipLaunchKernelGGL(k_batch_plan, dim3((count + kPlanWaves - 1) / kPlanWaves), dim3(64 * kPlanWaves), 0, st, d_desc,
                     count, B, dw, dub, dmm, plan, de, du, dh, dwords, err);
  PHOBIC_HIP(hipGetLastError());
  uint64_t *hwords, *ibase, *hdrs;  // pinned
  uint32_t* herr;
  PHOBIC_HIP(S.host(&hwords, (uint64_t)count));
  PHOBIC_HIP(S.host(&ibase, (uint64_t)count));
  PHOBIC_HIP(S.host(&hdrs, (uint64_t)count * kHeaderWords));
  PHOBIC_HIP(S.host(&herr, 6));
  PHOBIC_HIP(hipMemcpyAsync(hwords, dwords, (size_t)count * 8, hipMemcpyDeviceToHost, st));
  PHOBIC_HIP(hipMemcpyAsync(herr, err, 6 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  PHOBIC_HIP(spin_sync(st));
  if (herr[0] & ((1u << PHOBIC_E_DUPLICATE) | (1u << PHOBIC_E_PILOT_OVERFLOW))) {
    const uint64_t J = (uint64_t)herr[4] | ((uint64_t)herr[5] << 32);
    const uint32_t t = (uint32_t)(std::upper_bound(hKbase.begin(), hKbase.end(), J) - hKbase.begin()) - 1;
    const bool dup = herr[0] & (1u << PHOBIC_E_DUPLICATE);
    return fail(dup ? PHOBIC_E_DUPLICATE : PHOBIC_E_PILOT_OVERFLOW,
                "MPHF " + std::to_string(t) + (dup ? ": two keys share their hash code" : ": pilot overflow"));
  }
  if (herr[0] & (1u << PHOBIC_E_CAPACITY)) return fail(PHOBIC_E_CAPACITY, "a unary stream exceeds 2^32 bits");
  uint64_t total_words = 0;
  for (uint32_t t = 0; t < count; t++) {
    ibase[t] = total_words;
    total_words += hwords[t];
  }
  void* big = nullptr;
  PHOBIC_HIP(pool_alloc(&big, total_words * 8, st));
  std::shared_ptr<void> shared(big, [](void* p) { (void)hipFreeAsync(p, nullptr); });
  PHOBIC_HIP(hipMemcpyAsync(dib, ibase, (size_t)count * 8, hipMemcpyHostToDevice, st));
  uint64_t* bufw = (uint64_t*)big;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(total_words)), dim3(kBlock), 0, st, bufw, total_words, (uint64_t)0);
  hipLaunchKernelGGL(k_batch_heads, dim3(count), dim3(256), 0, st, dh, de, dib, B, bufw);
  hipLaunchKernelGGL(k_batch_pack_off, dim3(mphf_groups), dim3(256), 0, st, off, d_desc, count, dh, dib, bufw);
  hipLaunchKernelGGL(k_batch_pack_vals, dim3(item_groups), dim3(256), 0, st, pilots, d_desc, count, B, dh, de, du,
                     dib, bufw);
  if (prm.coding == PHOBIC_IC_RICE)
    hipLaunchKernelGGL(k_batch_sel_fill, dim3(count), dim3(256), 0, st, d_desc, B, dh, dib, bufw);
  PHOBIC_HIP(hipGetLastError());
  tm.mark();  // 4
  PHOBIC_HIP(hipMemcpyAsync(hdrs, dh, (size_t)count * kHeaderWords * 8, hipMemcpyDeviceToHost, st));
  PHOBIC_HIP(spin_sync(st));
  phobic_build_info info{};
  info.bucket_sort_ms = tm.ms(0, 1);  // hashing, partitioning and bucketing of all chunks
  info.search_ms = tm.ms(2, 3);
  info.encode_ms = tm.ms(3, 4);
  info.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_host0).count();
  info.max_partition_keys = hinfo[2];
  info.max_bucket_keys = hinfo[1];

  std::vector<phobic_mphf*> made(count, nullptr);
  for (uint32_t t = 0; t < count; t++) {
    phobic_mphf* h = new (std::nothrow) phobic_mphf();
    if (!h) {
      for (auto q : made) phobic_free(q);
      return fail(PHOBIC_E_OOM, "host allocation");
    }
    h->device = dev;
    h->n = desc[t].n;
    h->K = desc[t].K;
    h->B = B;
    h->prm = prm;
    h->d_table = tbl.d_table;
    h->d_image = bufw + ibase[t];
    h->header.assign(hdrs + (size_t)t * kHeaderWords, hdrs + (size_t)(t + 1) * kHeaderWords);
    h->nwords = h->header[kHWords];
    h->shared = shared;
    h->info = info;
    fill_query_args(h);
    made[t] = h;
  }
  for (uint32_t t = 0; t < count; t++) outs[t] = made[t];
  return PHOBIC_OK;
}

}  // namespace
}  // namespace phobic

using namespace phobic;

extern "C" phobic_status phobic_build_u64(const uint64_t* d_keys, uint64_t n, const phobic_params* params,
                                          void* hip_stream, phobic_mphf** out) {
  if (!out) return fail(PHOBIC_E_INVALID, "out is null");
  BuildInput in{Src::U64, d_keys, nullptr, nullptr, n};
  return build_impl(in, params, (hipStream_t)hip_stream, out, nullptr, nullptr);
}

extern "C" phobic_status phobic_build_str(const uint8_t* d_bytes, const uint64_t* d_offsets, uint64_t n,
                                          const phobic_params* params, void* hip_stream, phobic_mphf** out) {
  if (!out) return fail(PHOBIC_E_INVALID, "out is null");
  BuildInput in{Src::Str, nullptr, d_bytes, d_offsets, n};
  return build_impl(in, params, (hipStream_t)hip_stream, out, nullptr, nullptr);
}

extern "C" phobic_status phobic_partition_u64(const uint64_t* d_keys, uint64_t n, const phobic_params* params,
                                              void* hip_stream, uint64_t* d_offsets, uint64_t* d_codes) {
  if (!d_offsets || (n && !d_codes)) return fail(PHOBIC_E_INVALID, "null output pointer");
  BuildInput in{Src::U64, d_keys, nullptr, nullptr, n};
  return build_impl(in, params, (hipStream_t)hip_stream, nullptr, d_offsets, d_codes);
}

extern "C" phobic_status phobic_build_batch_u64(const uint64_t* const* h_key_ptrs, const uint64_t* h_counts,
                                                uint32_t count, const phobic_params* params, void* hip_stream,
                                                phobic_mphf** outs) {
  if (count && (!outs || !h_key_ptrs || !h_counts)) return fail(PHOBIC_E_INVALID, "null argument");
  for (uint32_t t = 0; t < count; t++) outs[t] = nullptr;
  if (count == 0) return PHOBIC_OK;
  return build_batch_impl(h_key_ptrs, h_counts, count, params, (hipStream_t)hip_stream, outs);
}
