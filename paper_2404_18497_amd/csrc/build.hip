// Construction of a PHOBIC MPHF on one MI355X (gfx950, wave64).
//
// Pipeline (one stream):
//   k_hash_count_*  : hash every key (a1) and histogram its partition j = mulhi(hi, K) (a2)
//   k_scan_offsets  : one workgroup: partition key offsets and table offsets (prefix sums, Sec. 4)
//   k_scatter_*     : hash again and scatter the 128-bit codes into their partition (order free)
//   k_bucket_sort   : one workgroup per partition: bucket of every key by the tabulated beta_eps
//                     (Sec. 3.1, Sec. 3.2, App. C.1), buckets ordered by size desc, index desc
//                     (Sec. 3, Sec. 5.1), keys rewritten in processing order
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
#include <cmath>
#include <cstring>
#include <vector>

#include "phobic_internal.h"

namespace phobic {
namespace {

constexpr int kBlock = 256;

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_u64(uint64_t* __restrict__ p, uint64_t n, uint64_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------------------------------------
// a1 + a2: hashing and partitioning
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
    atomicAdd(&cnt[__umul64hi(hi, K)], 1u);
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
// a3 + a4: bucket mapping and ordering, one workgroup (256 threads) per partition.
// LDS: cnt[nbpad] counts then start offsets, key[nbpad] sort keys (size << 16 | id), rec[n_j]
// per-key (bucket << 16 | rank in bucket).
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_bucket_sort(const ulonglong2* __restrict__ codes,
                                                        const uint64_t* __restrict__ off,
                                                        const uint64_t* __restrict__ T, uint32_t B, uint32_t nbpad,
                                                        ulonglong2* __restrict__ sorted, uint32_t* __restrict__ blist,
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
    sorted[base + cnt[r >> 16] + (r & 0xFFFF)] = codes[base + i];
  }
}

// ---------------------------------------------------------------------------------------------
// a5: pilot search, one wavefront per partition.
//
// F2 holds the free-slot bitmap twice in a row (bit t and bit t + m both mean "slot t is free"), so
// the 64 bits of displacements [d, d + 64) for a key at r are bits [r + d, r + d + 64) of F2 with no
// wrap-around.  For one seed s the lanes cover displacement windows d in [64 l, 64 l + 64); each key
// of the bucket ANDs its shifted window into the lane's accumulator; once every accumulator is zero
// no displacement of this seed works.  The lowest lane with a surviving bit holds the smallest d,
// which with s-major order is the smallest pilot.  Self-collisions under s are found first with a
// scratch bitmap and atomic OR; a collision at s = 0 also triggers the check for equal codes.
// ---------------------------------------------------------------------------------------------
struct SearchArgs {
  const ulonglong2* sorted;
  const uint64_t* off;
  const uint64_t* toff;
  const uint32_t* blist;
  const uint32_t* nbk;
  uint32_t* pilots;  // encoder-major: pilots[i * K + j]
  uint32_t* err;     // bit (1 << status) for every error met
  uint64_t* taken;   // global occupancy bitmap of all tables (alpha < 1), else null
  uint64_t K;
  uint64_t limit;
  uint32_t B;
  uint32_t f2_words, scr_words, rb_cap;
};

__device__ __forceinline__ uint64_t window64(const uint32_t* __restrict__ F2, uint32_t q) {
  uint32_t i = q >> 5, sh = q & 31;
  uint32_t w0 = F2[i], w1 = F2[i + 1], w2 = F2[i + 2];
  uint32_t lo = __builtin_amdgcn_alignbit(w1, w0, sh);
  uint32_t hi = __builtin_amdgcn_alignbit(w2, w1, sh);
  return ((uint64_t)hi << 32) | lo;
}

__global__ __launch_bounds__(64) void k_search(SearchArgs a) {
  extern __shared__ __align__(16) uint32_t lds[];
  uint32_t* F2 = lds;
  uint32_t* scr = lds + a.f2_words;
  uint16_t* rbuf = (uint16_t*)(scr + a.scr_words);
  uint64_t* cm = (uint64_t*)(rbuf + a.rb_cap);
  const uint32_t lane = threadIdx.x;
  const uint64_t j = blockIdx.x;
  const uint64_t kb = a.off[j];
  const uint32_t m = (uint32_t)(a.toff[j + 1] - a.toff[j]);
  const uint32_t twom = 2 * m;

  for (uint32_t w = lane; w < a.f2_words; w += 64) {
    uint32_t lo = w * 32;
    F2[w] = lo + 32 <= twom ? 0xFFFFFFFFu : (lo >= twom ? 0u : ((1u << (twom - lo)) - 1u));
  }
  for (uint32_t w = lane; w < a.scr_words; w += 64) scr[w] = 0;
  __syncthreads();

  const uint32_t nb = a.nbk[j];
  uint64_t kpos = kb;
  bool overflow = false;
  for (uint32_t r = 0; r < nb; r++) {
    const uint32_t e = a.blist[j * a.B + r];
    const uint32_t bid = e & 0xFFFF, sz = e >> 16;
    const ulonglong2* keys = a.sorted + kpos;
    kpos += sz;
    const uint32_t ng = (sz + 63) / 64;
    const ulonglong2 k0 = lane < sz ? keys[lane] : make_ulonglong2(0, 0);
    for (uint64_t s = 0;; s++) {
      // positions under seed s, and self-collisions
      bool coll_any = false;
      for (uint32_t g = 0; g < ng; g++) {
        const uint32_t k = g * 64 + lane;
        bool c = false;
        if (k < sz) {
          ulonglong2 key = g == 0 ? k0 : keys[k];
          uint32_t rr = pos_hash(key.x, key.y, s, m);
          rbuf[k] = (uint16_t)rr;
          uint32_t bit = 1u << (rr & 31);
          c = (atomicOr(&scr[rr >> 5], bit) & bit) != 0;
        }
        uint64_t bm = __ballot(c);
        if (lane == 0) cm[g] = bm;
        coll_any |= bm != 0;
      }
      __syncthreads();
      if (coll_any && s == 0) {
        // keys whose position repeats: an equal 128-bit code makes the bucket unplaceable
        bool dup = false;
        for (uint32_t g = 0; g < ng && !dup; g++) {
          uint64_t bm = cm[g];
          while (bm && !dup) {
            const uint32_t c = g * 64 + (uint32_t)(__ffsll((long long)bm) - 1);
            bm &= bm - 1;
            const uint32_t rc = rbuf[c];
            const ulonglong2 kc = keys[c];
            bool f = false;
            for (uint32_t k = lane; k < sz; k += 64) {
              if (k != c && rbuf[k] == rc) {
                ulonglong2 kk = keys[k];
                f |= kk.x == kc.x && kk.y == kc.y;
              }
            }
            dup = __ballot(f) != 0;
          }
        }
        if (dup) {
          if (lane == 0) atomicOr(a.err, 1u << PHOBIC_E_DUPLICATE);
          return;
        }
      }
      for (uint32_t k = lane; k < sz; k += 64) {
        uint32_t rr = rbuf[k];
        atomicAnd(&scr[rr >> 5], ~(1u << (rr & 31)));
      }
      __syncthreads();
      if (overflow) break;  // after an overflow only the duplicate check runs
      if (coll_any) continue;
      if (s * m > a.limit) {
        overflow = true;
        break;
      }

      // displacement scan: lowest d such that every key's slot (r + d) mod m is free
      uint32_t d_found = 0xFFFFFFFFu;
      for (uint32_t d0 = 0; d0 < m; d0 += 4096) {
        const uint32_t dl = d0 + lane * 64;
        uint64_t acc = 0;
        if (dl < m) acc = (m - dl >= 64) ? ~0ULL : ((1ULL << (m - dl)) - 1);
        for (uint32_t k = 0; k < sz; k += 4) {
          const uint64_t r4 = *(const uint64_t*)(rbuf + k);
#pragma unroll
          for (uint32_t t = 0; t < 4; t++) {
            if (k + t < sz && dl < m) acc &= window64(F2, (uint32_t)((r4 >> (16 * t)) & 0xFFFF) + dl);
          }
          if (__ballot(acc != 0) == 0) break;
        }
        const uint64_t bal = __ballot(acc != 0);
        if (bal) {
          const uint32_t L = (uint32_t)(__ffsll((long long)bal) - 1);
          const uint64_t accL = __shfl(acc, (int)L);
          d_found = d0 + L * 64 + (uint32_t)(__ffsll((long long)accL) - 1);
          break;
        }
      }
      if (d_found == 0xFFFFFFFFu) continue;
      const uint64_t p = s * m + d_found;
      if (p > a.limit) {
        overflow = true;
        break;
      }
      for (uint32_t k = lane; k < sz; k += 64) {
        uint32_t t = rbuf[k] + d_found;
        if (t >= m) t -= m;
        atomicAnd(&F2[t >> 5], ~(1u << (t & 31)));
        uint32_t t2 = t + m;
        atomicAnd(&F2[t2 >> 5], ~(1u << (t2 & 31)));
      }
      if (lane == 0) a.pilots[(uint64_t)bid * a.K + j] = (uint32_t)p;
      __syncthreads();
      break;
    }
  }
  if (overflow) {
    if (lane == 0) atomicOr(a.err, 1u << PHOBIC_E_PILOT_OVERFLOW);
    return;
  }
  if (a.taken) {
    const uint64_t tb = a.toff[j];
    for (uint32_t w = lane; w * 32 < m; w += 64) {
      uint32_t nbits = min(32u, m - w * 32);
      uint32_t busy = ~F2[w] & (nbits == 32 ? 0xFFFFFFFFu : ((1u << nbits) - 1));
      put_bits_atomic(a.taken, tb + (uint64_t)w * 32, busy, nbits);
    }
  }
}

// ---------------------------------------------------------------------------------------------
// a6: interleaved coding
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// One workgroup per encoder i: shsum[i * 33 + b] = sum_j (v_ij >> b), vmax[i] = max_j v_ij.
__global__ __launch_bounds__(kBlock) void k_encoder_stats(const uint32_t* __restrict__ pilots, uint64_t K,
                                                          uint64_t* __restrict__ shsum, uint32_t* __restrict__ vmax) {
  __shared__ uint64_t part[kBlock / 64][33];
  __shared__ uint32_t mx;
  const uint32_t tid = threadIdx.x, i = blockIdx.x;
  if (tid == 0) mx = 0;
  uint64_t acc[33];
#pragma unroll
  for (int b = 0; b < 33; b++) acc[b] = 0;
  uint32_t lmx = 0;
  const uint32_t* col = pilots + (uint64_t)i * K;
  for (uint64_t jj = tid; jj < K; jj += kBlock) {
    uint64_t v = col[jj];
    lmx = max(lmx, (uint32_t)v);
#pragma unroll
    for (int b = 0; b < 33; b++) acc[b] += v >> b;
  }
  __syncthreads();
  atomicMax(&mx, lmx);
#pragma unroll
  for (int b = 0; b < 33; b++) {
    uint64_t v = wave_sum_u64(acc[b]);
    if ((tid & 63) == 0) part[tid >> 6][b] = v;
  }
  __syncthreads();
  if (tid < 33) {
    uint64_t v = 0;
    for (int w = 0; w < kBlock / 64; w++) v += part[w][tid];
    shsum[(uint64_t)i * 33 + tid] = v;
  }
  if (tid == 0) vmax[i] = mx;
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
  atomicMin(&mm[0], lmin);
  atomicMax(&mm[1], lmax);
}

__global__ __launch_bounds__(kBlock) void k_pack_offsets(const uint64_t* __restrict__ toff, uint64_t K, uint64_t R,
                                                         long long dmin, uint32_t woff, uint64_t* __restrict__ sec) {
  for (uint64_t jj = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; jj <= K; jj += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t u = (uint64_t)((long long)(toff[jj] - expected_offset(jj, R)) - dmin);
    put_bits_atomic(sec, jj * woff, u, woff);
  }
}

// One workgroup of 1024 threads per encoder i: low bits (or Compact values) at base_i + j w_i; for
// Rice the unary stream of q = v >> w_i (q zeros then a one), whose one for value t = i K + j sits at
// ubase_i + sum_{j' < j} (q_j' + 1) + q_j, and a select sample for every 256th one.
constexpr int kPackThreads = 1024;
constexpr int kPackItems = 4;
__global__ __launch_bounds__(kPackThreads) void k_pack_values(const uint32_t* __restrict__ pilots, uint64_t K,
                                                              const uint64_t* __restrict__ enc,
                                                              const uint64_t* __restrict__ ubase, uint32_t rice,
                                                              uint64_t* __restrict__ data, uint64_t* __restrict__ unary,
                                                              uint32_t* __restrict__ sel) {
  __shared__ uint64_t part[kPackThreads / 64];
  __shared__ uint64_t chunk_total;
  const uint32_t tid = threadIdx.x, i = blockIdx.x;
  const uint64_t e = enc[i];
  const uint32_t w = (uint32_t)(e & 0xFF);
  const uint64_t base = e >> 8;
  const uint32_t* col = pilots + (uint64_t)i * K;
  uint64_t carry = rice ? ubase[i] : 0;
  for (uint64_t j0 = 0; j0 < K; j0 += (uint64_t)kPackThreads * kPackItems) {
    const uint64_t jb = j0 + (uint64_t)tid * kPackItems;
    uint64_t v[kPackItems];
    uint64_t local = 0;
#pragma unroll
    for (int t = 0; t < kPackItems; t++) {
      v[t] = jb + t < K ? col[jb + t] : 0;
      if (jb + t < K) local += (v[t] >> w) + 1;
    }
    uint64_t excl = 0;
    if (rice) {
      // block exclusive scan of local
      uint64_t incl = local;
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
      __syncthreads();
      excl = carry + part[tid >> 6] + (incl - local);
    }
#pragma unroll
    for (int t = 0; t < kPackItems; t++) {
      const uint64_t jj = jb + t;
      if (jj < K) {
        const uint64_t q = v[t] >> w;
        put_bits_atomic(data, base + jj * w, w >= 64 ? v[t] : (v[t] & ((1ULL << w) - 1)), w);
        if (rice) {
          const uint64_t pos = excl + q;
          atomicOr((unsigned long long*)&unary[pos >> 6], 1ULL << (pos & 63));
          const uint64_t t_glob = (uint64_t)i * K + jj;
          if ((t_glob & (kSelEvery - 1)) == 0) sel[t_glob / kSelEvery] = (uint32_t)pos;
          excl = pos + 1;
        }
      }
    }
    if (rice) {
      __syncthreads();
      carry += chunk_total;
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------------------------
// a8: remap for alpha < 1.  Table positions g >= n that hold a key, ascending, are paired with the
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

// exclusive scans of fc and oc in place, one workgroup
__global__ __launch_bounds__(1024) void k_scan_pair(uint32_t* __restrict__ fc, uint32_t* __restrict__ oc, uint64_t nw) {
  __shared__ uint64_t sf[1024], so[1024];
  const uint32_t t = threadIdx.x;
  const uint64_t per = (nw + 1023) / 1024;
  const uint64_t a = min(nw, (uint64_t)t * per), b = min(nw, a + per);
  uint64_t tf = 0, to = 0;
  for (uint64_t w = a; w < b; w++) { tf += fc[w]; to += oc[w]; }
  sf[t] = tf;
  so[t] = to;
  __syncthreads();
  for (uint32_t d = 1; d < 1024; d <<= 1) {
    uint64_t vf = t >= d ? sf[t - d] : 0, vo = t >= d ? so[t - d] : 0;
    __syncthreads();
    sf[t] += vf;
    so[t] += vo;
    __syncthreads();
  }
  uint64_t pf = sf[t] - tf, po = so[t] - to;
  for (uint64_t w = a; w < b; w++) {
    uint32_t f = fc[w], o = oc[w];
    fc[w] = (uint32_t)pf;
    oc[w] = (uint32_t)po;
    pf += f;
    po += o;
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

// Stream-ordered scratch allocations, released on every exit path.
struct Scratch {
  hipStream_t st;
  std::vector<void*> ptrs;
  explicit Scratch(hipStream_t s) : st(s) {}
  template <class T>
  hipError_t get(T** p, uint64_t count) {
    void* q = nullptr;
    hipError_t e = hipMallocAsync(&q, std::max<uint64_t>(count, 1) * sizeof(T), st);
    if (e == hipSuccess) ptrs.push_back(q);
    *p = (T*)q;
    return e;
  }
  ~Scratch() {
    for (void* p : ptrs) (void)hipFreeAsync(p, st);
  }
};

struct Timer {
  hipStream_t st;
  std::vector<hipEvent_t> ev;
  explicit Timer(hipStream_t s) : st(s) {}
  void mark() {
    hipEvent_t e;
    if (hipEventCreate(&e) == hipSuccess) {
      (void)hipEventRecord(e, st);
      ev.push_back(e);
    }
  }
  double ms(size_t a, size_t b) const {
    float t = 0;
    if (b < ev.size() && hipEventElapsedTime(&t, ev[a], ev[b]) != hipSuccess) return 0;
    return b < ev.size() ? t : 0;
  }
  ~Timer() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

void configure_pool_once() {
  static bool done = false;
  if (done) return;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  done = true;
}

enum class Src { U64, Str };

struct BuildInput {
  Src src;
  const uint64_t* keys;
  const uint8_t* bytes;
  const uint64_t* offs;
  uint64_t n;
};

phobic_status build_impl(const BuildInput& in, const phobic_params* params, hipStream_t st, phobic_mphf** out,
                         uint64_t* part_offsets_out, uint64_t* part_codes_out) {
  if (out) *out = nullptr;
  uint32_t B = 0;
  phobic_status vs = validate_params(params, &B);
  if (vs != PHOBIC_OK) return vs;
  if (B > kMaxBuckets)
    return fail(PHOBIC_E_CAPACITY, "B = ceil(P / lambda) = " + std::to_string(B) + " exceeds the device limit " +
                                       std::to_string(kMaxBuckets));
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

  uint32_t* cnt;
  uint64_t *off, *toff, *dinfo;
  ulonglong2 *codes, *stage = nullptr;
  PHOBIC_HIP(S.get(&cnt, K + 1));
  PHOBIC_HIP(S.get(&off, K + 1));
  PHOBIC_HIP(S.get(&toff, K + 1));
  PHOBIC_HIP(S.get(&dinfo, 8));
  PHOBIC_HIP(S.get(&codes, n));
  if (in.src == Src::Str) PHOBIC_HIP(S.get(&stage, n));
  std::vector<uint64_t> info(8, 0);

  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(K + 1)), dim3(kBlock), 0, st, cnt, K + 1, 0u);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, dinfo, (uint64_t)8, (uint64_t)0);
  tm.mark();  // 0
  if (in.src == Src::U64)
    hipLaunchKernelGGL(k_hash_count_u64, dim3(grid_for(n)), dim3(kBlock), 0, st, in.keys, n, prm.hash_seed, K, cnt);
  else
    hipLaunchKernelGGL(k_hash_count_str, dim3(grid_for(n)), dim3(kBlock), 0, st, in.bytes, in.offs, n, prm.hash_seed, K,
                       stage, cnt);
  tm.mark();  // 1
  hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(1024), 0, st, cnt, K, an, ad, off, toff, dinfo);
  tm.mark();  // 2
  PHOBIC_HIP(hipGetLastError());
  PHOBIC_HIP(hipMemcpyAsync(info.data(), dinfo, 3 * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
  PHOBIC_HIP(hipStreamSynchronize(st));
  const uint64_t max_nj = info[0], max_m = info[1], total = info[2];
  h->info.max_partition_keys = max_nj;
  if (max_nj > kMaxPartitionKeys || max_m > kMaxTableSlots)
    return fail(PHOBIC_E_CAPACITY, "a partition holds " + std::to_string(max_nj) + " keys (" + std::to_string(max_m) +
                                       " slots); the device path holds at most " +
                                       std::to_string(kMaxPartitionKeys) + " keys and " +
                                       std::to_string(kMaxTableSlots) + " slots per partition");

  if (in.src == Src::U64)
    hipLaunchKernelGGL(k_scatter_u64, dim3(grid_for(n)), dim3(kBlock), 0, st, in.keys, n, prm.hash_seed, K, off, cnt,
                       codes);
  else
    hipLaunchKernelGGL(k_scatter_codes, dim3(grid_for(n)), dim3(kBlock), 0, st, stage, n, K, off, cnt, codes);
  tm.mark();  // 3
  PHOBIC_HIP(hipGetLastError());

  if (part_offsets_out) {  // stages a1-a2 only
    PHOBIC_HIP(hipMemcpyAsync(part_offsets_out, off, (K + 1) * sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
    PHOBIC_HIP(hipMemcpyAsync(part_codes_out, codes, n * sizeof(ulonglong2), hipMemcpyDeviceToDevice, st));
    PHOBIC_HIP(hipStreamSynchronize(st));
    return PHOBIC_OK;
  }

  // a3 + a4
  ulonglong2* sorted;
  uint32_t *blist, *nbk, *pilots, *err, *maxb;
  PHOBIC_HIP(S.get(&sorted, n));
  PHOBIC_HIP(S.get(&blist, K * B));
  PHOBIC_HIP(S.get(&nbk, K));
  PHOBIC_HIP(S.get(&err, 4));
  maxb = err + 1;
  if (keep) {
    PHOBIC_HIP(hipMalloc(&h->d_pilots, std::max<uint64_t>(1, K * B) * sizeof(uint32_t)));
    pilots = h->d_pilots;
  } else {
    PHOBIC_HIP(S.get(&pilots, K * B));
  }
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(K * B)), dim3(kBlock), 0, st, pilots, K * B, 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, err, (uint64_t)4, 0u);
  const uint32_t nbpad = next_pow2(B);
  const size_t sort_lds = (2 * (size_t)nbpad + std::max<uint64_t>(max_nj, 1)) * sizeof(uint32_t);
  tm.mark();  // 4
  hipLaunchKernelGGL(k_bucket_sort, dim3((uint32_t)K), dim3(kBlock), sort_lds, st, codes, off, h->d_table, B, nbpad,
                     sorted, blist, nbk, maxb);
  tm.mark();  // 5
  PHOBIC_HIP(hipGetLastError());
  uint32_t hmaxb = 0;
  PHOBIC_HIP(hipMemcpyAsync(&hmaxb, maxb, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  PHOBIC_HIP(hipStreamSynchronize(st));
  h->info.max_bucket_keys = hmaxb;

  // a5
  uint64_t* taken = nullptr;
  const uint64_t taken_words = (total + 63) / 64 + 1;
  if (total > n) {
    PHOBIC_HIP(S.get(&taken, taken_words));
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(taken_words)), dim3(kBlock), 0, st, taken, taken_words,
                       (uint64_t)0);
  }
  SearchArgs sa;
  sa.sorted = sorted;
  sa.off = off;
  sa.toff = toff;
  sa.blist = blist;
  sa.nbk = nbk;
  sa.pilots = pilots;
  sa.err = err;
  sa.taken = taken;
  sa.K = K;
  sa.limit = limit;
  sa.B = B;
  const uint32_t mm = (uint32_t)std::max<uint64_t>(max_m, 1);
  sa.f2_words = (2 * mm + 127) / 32 + 1;
  sa.scr_words = (mm + 31) / 32 + 1;
  if ((sa.f2_words + sa.scr_words) & 1) sa.scr_words++;  // keeps rbuf 8-byte aligned
  sa.rb_cap = ((std::max<uint32_t>(hmaxb, 1) + 3) / 4) * 4 + 4;
  const uint32_t ngroups = (std::max<uint32_t>(hmaxb, 1) + 63) / 64;
  const size_t search_lds = (size_t)(sa.f2_words + sa.scr_words) * 4 + (size_t)sa.rb_cap * 2 + (size_t)ngroups * 8;
  tm.mark();  // 6
  hipLaunchKernelGGL(k_search, dim3((uint32_t)K), dim3(64), search_lds, st, sa);
  tm.mark();  // 7
  PHOBIC_HIP(hipGetLastError());

  // a6: statistics -> host parameters
  uint64_t* shsum;
  uint32_t* vmax;
  long long* dmm;
  PHOBIC_HIP(S.get(&shsum, (uint64_t)B * 33));
  PHOBIC_HIP(S.get(&vmax, B));
  PHOBIC_HIP(S.get(&dmm, 2));
  const uint64_t R = (uint64_t)(((unsigned __int128)total << 32) / K);
  const long long init_mm[2] = {LLONG_MAX, LLONG_MIN};
  PHOBIC_HIP(hipMemcpyAsync(dmm, init_mm, sizeof(init_mm), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_encoder_stats, dim3(B), dim3(kBlock), 0, st, pilots, K, shsum, vmax);
  hipLaunchKernelGGL(k_offset_stats, dim3(grid_for(K + 1)), dim3(kBlock), 0, st, toff, K, R, dmm);
  PHOBIC_HIP(hipGetLastError());
  std::vector<uint64_t> hsh((size_t)B * 33);
  std::vector<uint32_t> hmax(B);
  long long hmm[2];
  uint32_t herr = 0;
  PHOBIC_HIP(hipMemcpyAsync(hsh.data(), shsum, hsh.size() * 8, hipMemcpyDeviceToHost, st));
  PHOBIC_HIP(hipMemcpyAsync(hmax.data(), vmax, hmax.size() * 4, hipMemcpyDeviceToHost, st));
  PHOBIC_HIP(hipMemcpyAsync(hmm, dmm, sizeof(hmm), hipMemcpyDeviceToHost, st));
  PHOBIC_HIP(hipMemcpyAsync(&herr, err, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  PHOBIC_HIP(hipStreamSynchronize(st));
  if (herr & (1u << PHOBIC_E_DUPLICATE)) return fail(PHOBIC_E_DUPLICATE, "two keys share their 128-bit hash code");
  if (herr & (1u << PHOBIC_E_PILOT_OVERFLOW))
    return fail(PHOBIC_E_PILOT_OVERFLOW, "a bucket needs a pilot above " + std::to_string(limit));

  const bool rice = prm.coding == PHOBIC_IC_RICE;
  std::vector<uint64_t> enc(B), ubase(B);
  uint64_t data_bits = 0, unary_bits = 0;
  for (uint32_t i = 0; i < B; i++) {
    uint32_t w = rice ? rice_parameter(hsh[(size_t)i * 33], K) : bit_length(hmax[i]);
    enc[i] = (data_bits << 8) | w;
    data_bits += (uint64_t)w * K;
    if (rice) {
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
  const uint64_t nvals = K * B;
  const uint64_t nsel = rice ? (nvals + kSelEvery - 1) / kSelEvery : 0;
  std::vector<uint64_t> hdr(kHeaderWords, 0);
  hdr[kHMagic] = kMagic;
  hdr[kHN] = n;
  hdr[kHK] = K;
  hdr[kHB] = B;
  hdr[kHP] = prm.partition_size;
  std::memcpy(&hdr[kHLambda], &prm.lambda, 8);
  hdr[kHAlpha] = (uint64_t)an | ((uint64_t)ad << 32);
  hdr[kHCoding] = prm.coding;
  hdr[kHSeed] = prm.hash_seed;
  hdr[kHTotal] = total;
  hdr[kHDmin] = (uint64_t)dmin;
  hdr[kHWoff] = woff;
  hdr[kHSecOff] = kHeaderWords;
  hdr[kHSecEnc] = hdr[kHSecOff] + ((K + 1) * woff + 63) / 64 + 1;
  hdr[kHSecData] = hdr[kHSecEnc] + B + 1;
  hdr[kHSecUnary] = hdr[kHSecData] + (data_bits + 63) / 64 + 1;
  hdr[kHSecSel] = hdr[kHSecUnary] + (rice ? (unary_bits + 63) / 64 + 1 : 0);
  hdr[kHSecRemap] = hdr[kHSecSel] + (rice ? (nsel + 1) / 2 + 1 : 0);
  hdr[kHWremap] = wremap;
  hdr[kHNremap] = nremap;
  hdr[kHUbits] = rice ? unary_bits : 0;
  hdr[kHWords] = hdr[kHSecRemap] + (nremap ? (nremap * wremap + 63) / 64 + 1 : 0);
  hdr[kHR] = R;
  const uint64_t nwords = hdr[kHWords];

  PHOBIC_HIP(hipMalloc(&h->d_image, nwords * sizeof(uint64_t)));
  h->nwords = nwords;
  h->header = hdr;
  uint64_t* img = h->d_image;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(nwords)), dim3(kBlock), 0, st, img, nwords, (uint64_t)0);
  PHOBIC_HIP(hipMemcpyAsync(img, hdr.data(), kHeaderWords * 8, hipMemcpyHostToDevice, st));
  PHOBIC_HIP(hipMemcpyAsync(img + hdr[kHSecEnc], enc.data(), (size_t)B * 8, hipMemcpyHostToDevice, st));
  uint64_t* d_ubase = nullptr;
  if (rice) {
    PHOBIC_HIP(S.get(&d_ubase, B));
    PHOBIC_HIP(hipMemcpyAsync(d_ubase, ubase.data(), (size_t)B * 8, hipMemcpyHostToDevice, st));
  }
  if (woff)
    hipLaunchKernelGGL(k_pack_offsets, dim3(grid_for(K + 1)), dim3(kBlock), 0, st, toff, K, R, dmin, woff,
                       img + hdr[kHSecOff]);
  hipLaunchKernelGGL(k_pack_values, dim3(B), dim3(kPackThreads), 0, st, pilots, K, img + hdr[kHSecEnc], d_ubase,
                     (uint32_t)rice, img + hdr[kHSecData], img + hdr[kHSecUnary],
                     (uint32_t*)(img + hdr[kHSecSel]));
  PHOBIC_HIP(hipGetLastError());
  if (nremap && wremap) {
    uint32_t *fc, *oc, *freeslot;
    PHOBIC_HIP(S.get(&fc, taken_words));
    PHOBIC_HIP(S.get(&oc, taken_words));
    PHOBIC_HIP(S.get(&freeslot, nremap));
    hipLaunchKernelGGL(k_remap_count, dim3(grid_for(taken_words)), dim3(kBlock), 0, st, taken, taken_words, n, total,
                       fc, oc);
    hipLaunchKernelGGL(k_scan_pair, dim3(1), dim3(1024), 0, st, fc, oc, taken_words);
    hipLaunchKernelGGL(k_remap_free, dim3(grid_for(taken_words)), dim3(kBlock), 0, st, taken, taken_words, n, fc,
                       freeslot);
    hipLaunchKernelGGL(k_remap_fill, dim3(grid_for(nremap)), dim3(kBlock), 0, st, taken, n, total, oc, freeslot,
                       wremap, img + hdr[kHSecRemap]);
    PHOBIC_HIP(hipGetLastError());
  }
  tm.mark();  // 8
  PHOBIC_HIP(hipStreamSynchronize(st));
  auto t_host1 = std::chrono::steady_clock::now();

  h->info.hash_count_ms = tm.ms(0, 1);
  h->info.scan_ms = tm.ms(1, 2);
  h->info.scatter_ms = tm.ms(2, 3);
  h->info.bucket_sort_ms = tm.ms(4, 5);
  h->info.search_ms = tm.ms(6, 7);
  h->info.encode_ms = tm.ms(7, 8);
  h->info.total_ms = std::chrono::duration<double, std::milli>(t_host1 - t_host0).count();
  fill_query_args(h);
  *out = h;
  h = nullptr;  // ownership moves to the caller
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
