// Pilot search on the device: for every partition, the buckets in processing order get the
// smallest pilot whose positions are pairwise distinct and free (Sec. 4, Sec. 4.2, Alg. 1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <string>

#include "phobic_internal.h"
#include "search.h"

namespace phobic {
namespace {

__global__ void k_queue_reset(unsigned long long* q) {
  if (threadIdx.x == 0) *q = 0;
}

// ---------------------------------------------------------------------------------------------
// Pilot search, one wavefront per partition (wavefronts per workgroup set by the launch shape).
//
// F2 holds the free-slot bitmap twice in a row (bit t and bit t + m both mean "slot t is free", in
// 32-bit words), so the displacements [d, d + 64) of a key at position r are bits [r + d, r + d + 64)
// of F2 with no wrap-around.  For one seed the lanes cover displacement windows [64 l, 64 l + 64);
// each key of the bucket ANDs its shifted window into the lane's accumulator; when every
// accumulator is zero no displacement of this seed works.  The lowest lane with a surviving bit
// holds the smallest d, and seeds are tried in increasing order, so the first hit is the smallest
// pilot p = s m + d (Sec. 4; the same minimum as the sequential nested loop, Sec. 4.2).
//
// The key loop is pure vector/LDS work: positions are kept encoded as e = (r >> 5) << 18 | (r & 31),
// so the high half of e is the byte offset of the word holding bit r (added to the lane's offset
// straight from the high half, one instruction) and the low five bits are the funnel shift; the list is padded to a multiple of four with copies of its last entry (AND is
// idempotent), and lanes whose window lies beyond m read in-bounds words into an accumulator that
// is already zero.
//
// Two keys of a bucket at the same position under s rule out every d.  Buckets of more than
// kSmallBucket keys test this first (scratch bitmap, atomic OR); smaller ones find it while marking
// their slots (a slot already cleared by the same bucket) and undo the marks.  A repeat at s = 0
// between equal fingerprints means the bucket can never be placed: PHOBIC_E_DUPLICATE.
// ---------------------------------------------------------------------------------------------
constexpr uint32_t kSmallBucket = 24;



__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Values that are the same on every lane of the wavefront, moved to scalar registers so that the
// branches and loops that depend on them are scalar branches instead of exec-mask updates.
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  return ((uint64_t)uniform((uint32_t)(v >> 32)) << 32) | uniform((uint32_t)v);
}
__device__ __forceinline__ uint64_t lane_value64(uint64_t v, uint32_t lane) {
  return ((uint64_t)__builtin_amdgcn_readlane((uint32_t)(v >> 32), lane) << 32) |
         __builtin_amdgcn_readlane((uint32_t)v, lane);
}

// Encoded positions: the high half of a code is the byte offset, from F2, of the load that starts at
// the word holding bit r; the low five bits are r's funnel shift.  kShift (every path but the wide
// one): F2 is followed, x bytes on, by its copy shifted by one word, F2s (F2s word w = F2 word
// w + 1), and a position whose word index is odd is read from F2s, so that the load's first two
// words are one aligned 64-bit LDS read; the low half is then r itself (r < 2^16).
template <bool kShift>
struct PosCode {
  uint32_t x;
  __device__ __forceinline__ uint32_t enc(uint32_t r) const {
    if (!kShift) return ((r >> 5) << 18) | (r & 31);
    const uint32_t a = r >> 5;
    return ((4 * a + ((a & 1) ? x - 4 : 0u)) << 16) | r;
  }
  __device__ __forceinline__ uint32_t dec(uint32_t e) const {
    return kShift ? (e & 0xFFFFu) : (((e >> 18) << 5) | (e & 31));
  }
};

// Marks the positions of rbuf[0..sz) in the scratch bitmap; cm[g] gets the lanes of group g whose
// position was already marked.  Leaves the scratch clear.  Returns whether a position repeats.
template <class PC>
__device__ bool positions_repeat(const PC& pc, uint32_t* scr, const uint32_t* rbuf, uint32_t sz, uint64_t* cm,
                                 uint32_t lane) {
  bool any = false;
  const uint32_t ng = (sz + 63) >> 6;
  for (uint32_t g = 0; g < ng; g++) {
    const uint32_t k = g * 64 + lane;
    bool c = false;
    if (k < sz) {
      const uint32_t rr = pc.dec(rbuf[k]), bit = 1u << (rr & 31);
      c = (atomicOr(&scr[rr >> 5], bit) & bit) != 0;
    }
    const uint64_t bm = __ballot(c);
    if (lane == 0) cm[g] = bm;
    any |= bm != 0;
  }
  wave_sync();
  for (uint32_t k = lane; k < sz; k += 64) {
    const uint32_t rr = pc.dec(rbuf[k]);
    atomicAnd(&scr[rr >> 5], ~(1u << (rr & 31)));
  }
  wave_sync();
  return any;
}

// After positions_repeat: whether a repeated position comes from two equal fingerprints.
__device__ bool equal_fingerprints(const uint64_t* keys, const uint32_t* rbuf, uint32_t sz, const uint64_t* cm,
                                   uint32_t lane) {
  const uint32_t ng = (sz + 63) >> 6;
  for (uint32_t g = 0; g < ng; g++) {
    uint64_t bm = cm[g];
    while (bm) {
      const uint32_t c = g * 64 + (uint32_t)__builtin_ctzll(bm);
      bm &= bm - 1;
      const uint32_t rc = rbuf[c];
      const uint64_t fc = keys[c];
      bool f = false;
      for (uint32_t k = lane; k < sz; k += 64)
        if (k != c && rbuf[k] == rc) f |= keys[k] == fc;
      if (__ballot(f)) return true;
    }
  }
  return false;
}

// Positions of a bucket's keys under the seed value w, encoded into rbuf, padded to a multiple of
// eight with the last entry.  Returns lane k's position for k < 64 (the keys a small bucket marks).
template <class PC>
__device__ __forceinline__ uint32_t bucket_positions(const PC& pc, uint32_t* rbuf, const uint64_t* keys, uint64_t f0,
                                                     uint32_t sz, uint64_t w, uint32_t m, uint32_t lane) {
  const uint32_t szp = (sz + 7) & ~7u;
  // keys 0..63: every lane hashes (those past the bucket a neighbour's fingerprint, unused), so no
  // lane mask is set up; the padding lanes store the last key's position
  const uint32_t r0 = pos_hash(f0, w, m);
  if (sz <= 64) {
    const uint32_t last = __builtin_amdgcn_readlane(r0, sz - 1);
    if (lane < szp) rbuf[lane] = pc.enc(lane < sz ? r0 : last);
  } else {
    rbuf[lane] = pc.enc(r0);
    uint32_t r = 0, k = lane;
    for (uint32_t g = 1; g * 64 < sz; g++) {  // keys 64 and on
      k = g * 64 + lane;
      r = 0;
      if (k < sz) {
        r = pos_hash(keys[k], w, m);
        rbuf[k] = pc.enc(r);
      }
    }
    const uint32_t last = __builtin_amdgcn_readlane(r, (sz - 1) & 63);
    if (k >= sz && k < szp) rbuf[k] = pc.enc(last);
  }
  wave_sync();
  return r0;
}

// Positions of a big bucket's keys under the seed value w (keys 0..63 from f0, the lane's
// fingerprint), written to rbuf and marked in the scratch bitmap 64 keys at a time, stopping at the
// first group that repeats a position: most seeds of a big bucket repeat one within its first 64
// keys, and the rest need not be hashed.  Leaves the scratch clear; without a repeat rbuf is padded
// to a multiple of eight with the last entry.  Returns whether a position repeats.
template <class PC>
__device__ bool positions_repeat_early(const PC& pc, uint32_t* scr, uint32_t* rbuf, const uint64_t* keys, uint64_t f0,
                                       uint32_t sz, uint64_t w, uint32_t m, uint32_t lane) {
  bool rep = false;
  uint32_t g = 0, r = 0;
  for (; g * 64 < sz; g++) {
    const uint32_t k = g * 64 + lane;
    bool c = false;
    if (k < sz) {
      r = pos_hash(g == 0 ? f0 : keys[k], w, m);
      rbuf[k] = pc.enc(r);
      const uint32_t bit = 1u << (r & 31);
      c = (atomicOr(&scr[r >> 5], bit) & bit) != 0;
    }
    if (__ballot(c)) {
      rep = true;
      g++;
      break;
    }
  }
  wave_sync();
  const uint32_t marked = min(g * 64, sz);
  for (uint32_t k = lane; k < marked; k += 64) {
    const uint32_t rr = pc.dec(rbuf[k]);
    atomicAnd(&scr[rr >> 5], ~(1u << (rr & 31)));
  }
  if (!rep) {
    const uint32_t last = __builtin_amdgcn_readlane(r, (sz - 1) & 63);
    const uint32_t k = sz + lane;
    if (k < ((sz + 7) & ~7u)) rbuf[k] = pc.enc(last);
  }
  wave_sync();
  return rep;
}

// Argument fields that only the failure and output paths use, kept in LDS for the partition so that
// they need no registers during the bucket loops: error word, failing-partition word, pilots,
// owner, Kbase, Kt, occupancy bitmap, table offsets.
enum : uint32_t { kCtxErr, kCtxFail, kCtxPilots, kCtxOwner, kCtxKbase, kCtxKt, kCtxTaken, kCtxToff, kCtxWords };
static_assert(kCtxWords * 8 == kSearchCtxBytes, "context size");

__device__ __forceinline__ void note_failure(const uint64_t* ctx, uint64_t j, uint32_t status) {
  atomicOr((uint32_t*)ctx[kCtxErr], 1u << status);
  unsigned long long* fp = (unsigned long long*)ctx[kCtxFail];
  if (fp) atomicMin(fp, (unsigned long long)j);
}

// Places every bucket of partition j (global index).  Uniform across the wavefront.
//
// The buckets come in processing order, sizes non-increasing, so they fall into three runs that get
// their own loops: big buckets (more than kSmallBucket keys; positions checked for repeats before
// the scan), small ones (2 .. kSmallBucket keys; a repeat shows while marking) and single keys (no
// repeat possible; seed 0 always finds a free slot).  Seed-0 positions come from the fingerprint
// windows, hashed once per window instead of once per bucket, and the bucket list is read from
// global memory through 64-entry register windows.  kMulti: some table of the launch has more than
// 4096 slots, so a displacement scan may need several passes.  kWide: pilots are written to the
// global row directly and F2 has no shifted copy (partitions whose lists do not fit the LDS; one
// MPHF).
template <bool kMulti, bool kWide>
__device__ void search_partition(const SearchArgs& a, uint64_t j, uint32_t* F2, uint32_t lane) {
  constexpr bool kShift = !kWide;
  const uint64_t* const fpa = a.fp;
  const uint64_t* const offp = a.off;
  const uint64_t* const toffp = a.toff;
  const uint32_t* const blistp = a.blist;
  const uint32_t* const nbkp = a.nbk;
  const uint32_t f2_words = a.f2_words, scr_words = a.scr_words, bl_cap = a.bl_cap;
  const uint32_t B = a.B;
  uint32_t* const pilots_w = kWide ? a.pilots : nullptr;
  uint32_t* const F2s = F2 + f2_words;  // kShift: F2 shifted by one word
  uint32_t* scr = F2 + (kShift ? 2 : 1) * f2_words;
  uint32_t* rbuf = scr + scr_words;
  uint32_t* pil = rbuf + a.rb_cap;  // the partition's pilots, by bucket index
  uint64_t* cm = (uint64_t*)(pil + bl_cap);
  const PosCode<kShift> pc{4 * f2_words};
  uint64_t* ctx = cm + a.cm_cap;
  if (lane == 0) {
    ctx[kCtxErr] = (uint64_t)a.err;
    ctx[kCtxFail] = (uint64_t)a.fail_part;
    ctx[kCtxPilots] = (uint64_t)a.pilots;
    ctx[kCtxOwner] = (uint64_t)a.owner;
    ctx[kCtxKbase] = (uint64_t)a.Kbase;
    ctx[kCtxKt] = (uint64_t)a.Kt;
    ctx[kCtxTaken] = (uint64_t)a.taken;
    ctx[kCtxToff] = (uint64_t)a.toff;
  }
  wave_sync();

  const uint64_t kb = uniform64(offp[j]);
  const uint32_t m = uniform((uint32_t)(toffp[j + 1] - toffp[j]));
  {  // the LDS layout was sized from bounds: a larger table or bucket is left to an exact resize
    const uint32_t nb0 = uniform(nbkp[j]);
    const uint32_t big0 = nb0 ? uniform(blistp[j * B]) >> 16 : 0u;
    if (m > a.max_m || big0 > a.max_bucket) {
      if (lane == 0) note_failure(ctx, j, kErrResize);
      return;
    }
  }
  const uint32_t twom = 2 * m;
  auto f2_init = [&](uint32_t w) -> uint32_t {  // word w of F2 with every slot free
    const uint32_t lo = w * 32;
    return lo + 32 <= twom ? 0xFFFFFFFFu : (lo >= twom ? 0u : ((1u << (twom - lo)) - 1u));
  };
  for (uint32_t w = lane; w < f2_words; w += 64) {
    F2[w] = f2_init(w);
    if (kShift) F2s[w] = f2_init(w + 1);
  }
  for (uint32_t w = lane; w < scr_words; w += 64) scr[w] = 0;
  const uint32_t nb = uniform(nbkp[j]);
  const uint32_t* gbl = blistp + j * B;
  // the bucket list: entries bbase + lane (bw0) and bbase + 64 + lane (bw1)
  uint32_t bw0 = lane < nb ? gbl[lane] : 0u, bw1 = 64 + lane < nb ? gbl[64 + lane] : 0u, bbase = 0;
  if (kWide) {
    for (uint32_t x = lane; x < B; x += 64) pilots_w[j * B + x] = 0;  // empty buckets keep pilot 0
    __threadfence_block();  // the zeros land before any pilot of this row
  } else {
    for (uint32_t x = lane; x < B; x += 64) pil[x] = 0;  // empty buckets keep pilot 0
  }
  wave_sync();
  const char* F2b = (const char*)F2;
  // the 64 bits of F2 from bit (off's word) * 32 + sh on: one aligned 64-bit read and one 32-bit
  // read (kShift), else three 32-bit reads
  auto window = [&](uint32_t off, uint32_t sh) -> uint64_t {
    const char* p = F2b + off;
    uint32_t w0, w1;
    if (kShift) {
      const uint2 q = *(const uint2*)p;
      w0 = q.x;
      w1 = q.y;
    } else {
      w0 = ((const uint32_t*)p)[0];
      w1 = ((const uint32_t*)p)[1];
    }
    const uint32_t w2 = ((const uint32_t*)p)[2];
    return ((uint64_t)__builtin_amdgcn_alignbit(w2, w1, sh) << 32) | __builtin_amdgcn_alignbit(w1, w0, sh);
  };
  // marks slot bit t (t < 2m) of F2 taken, and its copy in F2s, word (t >> 5) - 1 there: for t < 32
  // that is F2's last word, which lies past every window read (padding), so no test is needed
  auto take_bit = [&](uint32_t t) {
    uint32_t* const w = F2 + (t >> 5);
    const uint32_t mask = ~(1u << (t & 31));
    atomicAnd(w, mask);
    if (kShift) atomicAnd(w + (f2_words - 1), mask);
  };
  // bucket entry r (size << 16 | bucket) of the processing order; r never decreases
  auto bucket_entry = [&](uint32_t r) -> uint32_t {
    if (r >= bbase + 64) {
      bbase += 64;
      bw0 = bw1;
      bw1 = bbase + 64 + lane < nb ? gbl[bbase + 64 + lane] : 0u;
    }
    return __builtin_amdgcn_readlane(bw0, r - bbase);
  };
  // every lane calls it: the LDS row takes the same value from all of them, the global row (wide
  // partitions) from lane 0
  auto set_pilot = [&](uint32_t bid, uint32_t p) {
    if (kWide) {
      if (lane == 0) pilots_w[j * B + bid] = p;
    } else {
      pil[bid] = p;
    }
  };

  // this lane's displacement window of the first pass (d0 = 0): its bits below m, its byte offset
  const uint32_t dl0 = lane * 64;
  const uint64_t acc_first = dl0 < m ? (m - dl0 >= 64 ? ~0ULL : ((1ULL << (m - dl0)) - 1)) : 0ULL;
  const uint32_t loff_first = dl0 < m ? (dl0 >> 3) : 0u;

  const uint32_t nj = uniform((uint32_t)(offp[j + 1] - kb));
  // s m > limit exactly when s > floor(limit / m); limit < 2^32, so every seed tried fits 32 bits.
  // The cap at 2^32 - 2 (which only m = 1 reaches, where the one key takes seed 0) keeps s + 1 from
  // wrapping.
  const uint32_t smax = uniform(m ? (uint32_t)min<uint64_t>(a.limit / m, 0xFFFFFFFEULL) : 0u);
  const uint32_t dlast = uniform(m ? (uint32_t)(a.limit - smax * m) : 0);  // largest d allowed with s = smax

  // Fingerprints arrive through a sliding window: lane l of win0 holds key wbase + l of the partition
  // (processing order), win1 the next 64.  The keys of consecutive buckets are consecutive, so one
  // load serves many small buckets, and the next window is in flight while the current one is used.
  // p0w0 holds win0's positions under seed 0; p0w1 win1's once a bucket has needed them (p1).
  uint32_t wbase = 0, o = 0;  // o: first key of the current bucket
  uint64_t win0 = lane < nj ? fpa[kb + lane] : 0;
  uint64_t win1 = 64 + lane < nj ? fpa[kb + 64 + lane] : 0;
  uint32_t p0w0 = pos_hash(win0, kPhi64, m), p0w1 = 0;
  bool p1 = false;
  // Moves the windows so that the bucket starting at key o lies in them (its first 64 keys).
  auto advance = [&]() {
    if (o >= wbase + 64) {
      if (o < wbase + 128) {
        win0 = win1;
        p0w0 = p1 ? p0w1 : pos_hash(win0, kPhi64, m);
        wbase += 64;
      } else {  // past both windows (after a big bucket)
        wbase = o;
        win0 = wbase + lane < nj ? fpa[kb + wbase + lane] : 0;
        p0w0 = pos_hash(win0, kPhi64, m);
      }
      win1 = wbase + 64 + lane < nj ? fpa[kb + wbase + 64 + lane] : 0;
      p1 = false;
    }
  };
  // key o + lane's fingerprint (lanes past the bucket get a neighbour's, unused)
  auto key_fp_at = [&](uint32_t ob, uint32_t sz) -> uint64_t {
    const uint32_t widx = ob - wbase + lane;
    const uint64_t f0a = __shfl(win0, (int)(widx & 63));
    if (uniform(ob - wbase + sz) <= 64) return f0a;
    const uint64_t f0b = __shfl(win1, (int)(widx & 63));
    return widx < 64 ? f0a : f0b;
  };
  auto key_fp = [&](uint32_t sz) -> uint64_t { return key_fp_at(o, sz); };
  // key o + lane's position under seed 0, for a bucket of sz keys
  auto key_p0 = [&](uint32_t sz) -> uint32_t {
    if (o - wbase + sz > 64 && !p1) {  // the bucket reaches into win1
      p0w1 = pos_hash(win1, kPhi64, m);
      p1 = true;
    }
    const uint32_t widx = o - wbase + lane;
    const uint32_t pa = __shfl(p0w0, (int)(widx & 63));
    if (uniform(o - wbase + sz) <= 64) return pa;
    const uint32_t pb = __shfl(p0w1, (int)(widx & 63));
    return widx < 64 ? pa : pb;
  };

  // displacement scan: the lowest d such that every key's slot (r + d) mod m is free, for the szp
  // encoded positions at rb.  A pass covers 4096 displacements from d0 (acc: this lane's window
  // bits below m, loff: its byte offset); the first pass covers every m up to 4096, further passes
  // (kMulti) the larger ones.  ~0 when no displacement works.
  // ANDs the windows of the szp encoded positions at rb (this lane's list; szp >= 4, a multiple of
  // four) into acc, four keys at a time while some lane's window still has a bit; returns the
  // ballot of the lanes with one.
  auto keys_and = [&](const uint32_t* rb, uint64_t& acc, uint32_t loff, uint32_t szp) -> uint64_t {
    auto four = [&](uint32_t k) {
      const uint4 e4 = *(const uint4*)(rb + k);
      const uint32_t ev[4] = {e4.x, e4.y, e4.z, e4.w};
#pragma unroll
      for (int t = 0; t < 4; t++) acc &= window((ev[t] >> 16) + loff, ev[t]);
      return uniform64(__ballot(acc != 0));
    };
    uint64_t bal = four(0);
    for (uint32_t k = 4; bal != 0 && k < szp; k += 4) bal = four(k);
    return bal;
  };
  auto scan = [&](const uint32_t* rb, uint32_t szp) -> uint32_t {
    uint32_t d_found = 0xFFFFFFFFu;
    auto scan_pass = [&](uint32_t d0, uint64_t acc, uint32_t loff) {
      const uint64_t bal = keys_and(rb, acc, loff, szp);
      if (bal) {
        const uint32_t L = (uint32_t)__builtin_ctzll(bal);
        const uint64_t accL = lane_value64(acc, L);
        d_found = d0 + L * 64 + (uint32_t)__builtin_ctzll(accL);
      }
    };
    scan_pass(0, acc_first, loff_first);
    if (kMulti) {
      for (uint32_t d0 = 4096; d_found == 0xFFFFFFFFu && d0 < m; d0 += 4096) {
        const uint32_t dl = d0 + dl0;
        const bool act = dl < m;
        scan_pass(d0, act ? (m - dl >= 64 ? ~0ULL : ((1ULL << (m - dl)) - 1)) : 0ULL, act ? (dl >> 3) : 0u);
      }
    }
    return d_found;
  };

  // Short scan for big buckets early in the partition: the lanes form 8 windows of 64 displacements
  // (d < 512) times 8 key groups (lane = 8 g + w); group g ANDs every eighth key of the bucket into
  // its windows and the groups' windows are ANDed together at the end, so a step covers eight keys.
  // Returns the lowest d < 512, or ~0 when none is admissible there (the full scan then runs).
  const uint32_t gw = lane & 7, gg = lane >> 3;
  const uint64_t acc8 = 64 * gw < m ? (m - 64 * gw >= 64 ? ~0ULL : ((1ULL << (m - 64 * gw)) - 1)) : 0ULL;
  const uint32_t loff8 = 64 * gw < m ? gw * 8 : 0u;
  auto scan8 = [&](uint32_t szp8) -> uint32_t {
    uint64_t acc = acc8;
    for (uint32_t k = 0;;) {
      const uint32_t e = rbuf[k + gg];
      acc &= window((e >> 16) + loff8, e);
      k += 8;
      if (k >= szp8) break;
      // a key group with all eight windows empty empties the AND: some byte of the ballot is zero
      const uint64_t b = uniform64(__ballot(acc != 0));
      if (((b - 0x0101010101010101ULL) & ~b & 0x8080808080808080ULL) != 0) return 0xFFFFFFFFu;
    }
    acc &= __shfl_xor(acc, 8);
    acc &= __shfl_xor(acc, 16);
    acc &= __shfl_xor(acc, 32);
    const uint64_t b = uniform64(__ballot(acc != 0)) & 0xFFull;
    if (!b) return 0xFFFFFFFFu;
    const uint32_t L = (uint32_t)__builtin_ctzll(b);
    return L * 64 + (uint32_t)__builtin_ctzll(lane_value64(acc, L));
  };
  uint32_t placed = 0;  // keys placed so far

  bool overflow = false;
  uint32_t r = 0;
  const uint64_t* keys = fpa + kb;  // the current bucket's keys

  // ---- big buckets: every seed's positions are checked for repeats first --------------------
  for (; r < nb; r++) {
    const uint32_t e = bucket_entry(r);
    const uint32_t bid = e & 0xFFFF, sz = e >> 16;
    if (sz <= kSmallBucket) break;
    advance();
    keys = fpa + kb + o;
    const uint64_t f0 = key_fp(sz);
    o += sz;
    uint64_t wseed = kPhi64;  // the seed's Weyl value (s + 1) phi, kept as a running sum
    for (uint32_t s = 0;; s++, wseed += kPhi64) {
      if (s > smax) {  // every pilot s m + d of this seed exceeds the limit
        overflow = true;
        break;
      }
      if (s == 0) {  // all positions, for the duplicate check
        bucket_positions(pc, rbuf, keys, f0, sz, wseed, m, lane);
        if (positions_repeat(pc, scr, rbuf, sz, cm, lane)) {
          if (equal_fingerprints(keys, rbuf, sz, cm, lane)) {
            if (lane == 0) note_failure(ctx, j, PHOBIC_E_DUPLICATE);
            return;
          }
          continue;
        }
      } else if (positions_repeat_early(pc, scr, rbuf, keys, f0, sz, wseed, m, lane)) {
        continue;
      }
      // the short scan first while the bucket expects at least three admissible displacements below
      // 512 (512 f^sz >= 3 for the free fraction f); the choice only decides which scan runs first
      uint32_t d_found = 0xFFFFFFFFu;
      if (m > 512 && (float)sz * __logf((float)(m - placed) / (float)m) >= -5.14f) d_found = scan8((sz + 7) & ~7u);
      if (d_found == 0xFFFFFFFFu) d_found = scan(rbuf, (sz + 3) & ~3u);
      if (d_found == 0xFFFFFFFFu) continue;
      if (s == smax && d_found > dlast) {  // p > limit, with s <= smax
        overflow = true;
        break;
      }
      for (uint32_t k = lane; k < sz; k += 64) {
        uint32_t t = pc.dec(rbuf[k]) + d_found;
        if (t >= m) t -= m;
        take_bit(t);
        take_bit(t + m);
      }
      set_pilot(bid, s * m + d_found);
      placed += sz;
      wave_sync();
      break;
    }
    if (overflow) {
      r++;
      break;
    }
  }

  // ---- small buckets (2 .. kSmallBucket keys): a repeat shows while marking ------------------
  // Seed 0 takes its positions from the fingerprint window.  Later seeds are hashed G at a time:
  // the lanes form G groups of S lanes (S the smallest of 4, 8, 16, 32 that holds the bucket), lane
  // x holding key x mod S (the last key past the bucket) under seed s + x / S, so one hash evaluation
  // serves G seeds; group i's positions are entries i S .. i S + S of rbuf.
  // windows of 64 displacements per seed, and lane x's place in them: window x mod NW of seed x / NW
  const uint32_t NW = (m + 63) >> 6;
  const uint32_t lane_q = NW ? lane / NW : 0u, lane_r = lane - lane_q * NW;
  const uint32_t q64 = NW ? 64u / NW : 0u, r64 = 64u - q64 * NW;
  if (!overflow) {
    for (; r < nb; r++) {
      const uint32_t e = bucket_entry(r);
      const uint32_t bid = e & 0xFFFF, sz = e >> 16;
      if (sz < 2) break;
      advance();
      const uint32_t ob = o;
      keys = fpa + kb + o;
      o += sz;
      const uint32_t szp = (sz + 3) & ~3u;
      // marks the slots of the keys (lane k < sz: key k at position pos) for displacement d; false
      // (and the table unchanged) when two of them share a slot
      auto place = [&](uint32_t pos, uint32_t d) -> bool {
        uint32_t t = pos + d;
        if (t >= m) t -= m;
        bool mine = true;
        if (lane < sz) mine = (atomicAnd(&F2[t >> 5], ~(1u << (t & 31))) >> (t & 31)) & 1u;
        wave_sync();
        if (uniform64(__ballot(!mine))) {
          if (lane < sz && mine) atomicOr(&F2[t >> 5], 1u << (t & 31));  // undo
          wave_sync();
          return false;
        }
        if (lane < sz) {
          if (kShift) atomicAnd(&F2[(t >> 5) + (f2_words - 1)], ~(1u << (t & 31)));  // F2s, see take_bit
          take_bit(t + m);
        }
        return true;
      };
      auto dup0 = [&]() -> bool {  // after a failure at seed 0 (positions in rbuf): equal keys?
        return positions_repeat(pc, scr, rbuf, sz, cm, lane) && equal_fingerprints(keys, rbuf, sz, cm, lane);
      };
      // seed 0
      {
        const uint32_t widx = ob - wbase + (lane < sz ? lane : sz - 1);
        const uint32_t pa = __shfl(p0w0, (int)(widx & 63));
        uint32_t p0 = pa;
        if (uniform(ob - wbase + sz) > 64) {
          if (!p1) {
            p0w1 = pos_hash(win1, kPhi64, m);
            p1 = true;
          }
          const uint32_t pb = __shfl(p0w1, (int)(widx & 63));
          p0 = widx < 64 ? pa : pb;
        }
        rbuf[lane] = pc.enc(p0);
        wave_sync();
        const uint32_t d = scan(rbuf, szp);
        const bool in_limit = d != 0xFFFFFFFFu && !(smax == 0 && d > dlast);
        if (in_limit && place(p0, d)) {
          set_pilot(bid, d);
          wave_sync();
          continue;
        }
        if (dup0()) {
          if (lane == 0) note_failure(ctx, j, PHOBIC_E_DUPLICATE);
          return;
        }
        if (smax == 0) {
          overflow = true;
          r++;
          break;
        }
      }
      // seeds 1, 2, ...: G at a time
      const uint32_t lgS = sz <= 4 ? 2u : (sz <= 8 ? 3u : (sz <= 16 ? 4u : 5u));
      const uint32_t S = 1u << lgS, G = 64u >> lgS;
      const uint32_t kx = lane & (S - 1);
      uint64_t fS;  // fingerprint of key min(kx, sz - 1) of the bucket
      {
        const uint32_t widx = ob - wbase + (kx < sz ? kx : sz - 1);
        const uint64_t fa = __shfl(win0, (int)(widx & 63));
        fS = fa;
        if (uniform(ob - wbase + sz) > 64) {
          const uint64_t fb = __shfl(win1, (int)(widx & 63));
          fS = widx < 64 ? fa : fb;
        }
      }
      // Weyl value of this lane's seed, (s + 1 + x / S) phi, advanced by G phi per batch
      uint64_t wl = (uint64_t)(2 + (lane >> lgS)) * kPhi64;
      const uint64_t gstep = (uint64_t)G * kPhi64;
      bool done = false;
      if (!kMulti) {
        // The batch's G seeds times NW windows of 64 displacements, in pilot order (seed, then
        // window), are scanned 64 windows at a time: lane x of chunk c takes window c 64 + x, so
        // every lane has a window instead of the NW of one seed.  The lowest surviving lane holds
        // the smallest pilot of the chunk; a seed whose positions repeat (marking fails) drops out.
        const uint32_t nwin = G * NW;
        for (uint32_t s = 1; !done; s += G, wl += gstep) {
          rbuf[lane] = pc.enc(pos_hash(fS, wl, m));
          wave_sync();
          uint32_t t0 = 0, r0 = 0;  // chunk c starts at seed t0 of the batch, window r0
          for (uint32_t c = 0; c < nwin; c += 64) {
            uint32_t dw = r0 + lane_r, t = t0 + lane_q;
            if (dw >= NW) {
              dw -= NW;
              t++;
            }
            const uint32_t dlo = dw * 64;
            const bool act = t < G && s + t <= smax;
            uint64_t acc = act ? (m - dlo >= 64 ? ~0ULL : ((1ULL << (m - dlo)) - 1)) : 0ULL;
            uint64_t bal = keys_and(rbuf + (act ? t * S : 0u), acc, act ? dw * 8 : 0u, szp);
            while (bal) {
              const uint32_t L = (uint32_t)__builtin_ctzll(bal);
              const uint32_t tL = __builtin_amdgcn_readlane(t, L);
              const uint32_t d = __builtin_amdgcn_readlane(dlo, L) + (uint32_t)__builtin_ctzll(lane_value64(acc, L));
              const uint32_t sd = s + tL;
              if (sd == smax && d > dlast) {
                overflow = true;
                break;
              }
              if (place(pc.dec(rbuf[tL * S + (lane < sz ? lane : 0u)]), d)) {
                set_pilot(bid, sd * m + d);
                wave_sync();
                done = true;
                break;
              }
              bal &= ~uniform64(__ballot(t == tL));
            }
            if (done || overflow) break;
            t0 += q64;
            r0 += r64;
            if (r0 >= NW) {
              r0 -= NW;
              t0++;
            }
          }
          if (!done && s + G - 1 >= smax) overflow = true;  // every seed up to smax was tried
          if (overflow) break;
        }
      }
      for (uint32_t s = 1; kMulti && !done; s += G, wl += gstep) {
        rbuf[lane] = pc.enc(pos_hash(fS, wl, m));
        wave_sync();
        for (uint32_t i = 0; i < G; i++) {
          const uint32_t sd = s + i;
          if (sd > smax) {
            overflow = true;
            break;
          }
          const uint32_t* rb = rbuf + i * S;
          const uint32_t d = scan(rb, szp);
          if (d == 0xFFFFFFFFu) continue;
          if (sd == smax && d > dlast) {
            overflow = true;
            break;
          }
          if (!place(pc.dec(rb[lane < sz ? lane : 0u]), d)) continue;
          set_pilot(bid, sd * m + d);
          wave_sync();
          done = true;
          break;
        }
        if (overflow) break;
      }
      if (overflow) {
        r++;
        break;
      }
    }
  }

  // ---- single keys: seed 0, the first free slot at or after the key's position ---------------
  if (!overflow) {
    for (; r < nb; r++) {
      const uint32_t bid = bucket_entry(r) & 0xFFFF;
      advance();
      const uint32_t r0 = __builtin_amdgcn_readlane(p0w0, o - wbase);
      o += 1;
      const uint32_t ebase = pc.enc(r0) >> 16;  // byte offset of the load at the word holding bit r0
      uint32_t d_found = 0xFFFFFFFFu;
      auto single_pass = [&](uint32_t d0, uint64_t acc, uint32_t loff) {
        acc &= window(ebase + loff, r0);
        const uint64_t bal = __ballot(acc != 0);
        if (bal) {
          const uint32_t L = (uint32_t)__builtin_ctzll(bal);
          const uint64_t accL = lane_value64(acc, L);
          d_found = d0 + L * 64 + (uint32_t)__builtin_ctzll(accL);
        }
      };
      single_pass(0, acc_first, loff_first);
      if (kMulti) {
        for (uint32_t d0 = 4096; d_found == 0xFFFFFFFFu && d0 < m; d0 += 4096) {
          const uint32_t dl = d0 + dl0;
          const bool act = dl < m;
          single_pass(d0, act ? (m - dl >= 64 ? ~0ULL : ((1ULL << (m - dl)) - 1)) : 0ULL, act ? (dl >> 3) : 0u);
        }
      }
      // a free slot always exists (fewer keys placed than slots), so d_found < m
      if (smax == 0 && d_found > dlast) {  // the pilot d exceeds the limit
        overflow = true;
        r++;
        break;
      }
      uint32_t t = r0 + d_found;
      if (t >= m) t -= m;
      if (lane < 4) {  // lane 0 the slot's bit, lane 1 its copy m bits further; lanes 2, 3 those of F2s
        const uint32_t tt = t + (lane & 1) * m;
        if (lane < 2) {
          atomicAnd(&F2[tt >> 5], ~(1u << (tt & 31)));
          set_pilot(bid, d_found);
        } else if (kShift) {  // F2s, see take_bit
          atomicAnd(&F2[(tt >> 5) + (f2_words - 1)], ~(1u << (tt & 31)));
        }
      }
      wave_sync();
    }
  }

  if (overflow) {  // the partition has failed: only look for equal fingerprints in the rest
    for (; r < nb; r++) {
      const uint32_t sz = bucket_entry(r) >> 16;
      advance();
      keys = fpa + kb + o;
      const uint64_t f0 = key_fp(sz);
      o += sz;
      if (sz < 2) continue;
      bucket_positions(pc, rbuf, keys, f0, sz, kPhi64, m, lane);
      if (positions_repeat(pc, scr, rbuf, sz, cm, lane) && equal_fingerprints(keys, rbuf, sz, cm, lane)) {
        if (lane == 0) note_failure(ctx, j, PHOBIC_E_DUPLICATE);
        return;
      }
    }
    if (lane == 0) note_failure(ctx, j, PHOBIC_E_PILOT_OVERFLOW);
    return;
  }
  wave_sync();
  uint32_t* const pilots = (uint32_t*)uniform64(ctx[kCtxPilots]);
  const uint32_t* const owner = (const uint32_t*)uniform64(ctx[kCtxOwner]);
  if (kWide) {
    // the pilots are in place
  } else if (owner) {  // several MPHFs: MPHF t's pilots, encoder-major, at B Kbase_t (zero-filled before)
    const uint32_t t = owner[j];
    const uint64_t jb = ((const uint64_t*)uniform64(ctx[kCtxKbase]))[t], kt = ((const uint64_t*)uniform64(ctx[kCtxKt]))[t];
    for (uint32_t x = lane; x < B; x += 64) {
      const uint32_t v = pil[x];
      if (v) pilots[(uint64_t)B * jb + (uint64_t)x * kt + (j - jb)] = v;
    }
  } else {  // one MPHF: row j of the partition-major array, written whole
    for (uint32_t x = lane; x < B; x += 64) pilots[j * B + x] = pil[x];
  }
  uint64_t* const taken = (uint64_t*)uniform64(ctx[kCtxTaken]);
  if (taken) {
    const uint64_t tb = ((const uint64_t*)uniform64(ctx[kCtxToff]))[j];
    for (uint32_t w = lane; w * 32 < m; w += 64) {
      const uint32_t nbits = min(32u, m - w * 32);
      const uint32_t busy = ~F2[w] & (nbits == 32 ? 0xFFFFFFFFu : ((1u << nbits) - 1));
      put_bits_atomic(taken, tb + (uint64_t)w * 32, busy, nbits);
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Launch order.  A partition's search time is dominated by per-bucket work (about proportional to
// its buckets and keys) plus the seeds its biggest buckets need before their positions stop
// repeating, about exp(k (k - 1) / (2 m)) for a bucket of k keys in m slots.  Starting the costly
// partitions first shortens the tail of the launch, where fewer and fewer wavefronts run.  The
// estimate is binned on a log scale (kOrderBins bins, 16 per octave) and the partitions are
// counting-sorted by bin, largest first; the order inside a bin is arbitrary.
// ---------------------------------------------------------------------------------------------
constexpr uint32_t kOrderBins = 256;
constexpr uint32_t kOrderThreads = 1024;
constexpr uint32_t kOrderPer = 4;  // partitions per thread of k_order_scatter

// The estimate's bin for partition j, computed by the 64 lanes of a wavefront: lane x adds the
// terms of the buckets x, x + 64, ... of the list (coalesced reads), stopping after the first
// window of 64 that reaches buckets of fewer than 8 keys (sizes are non-increasing).  Uniform.
__device__ __forceinline__ uint32_t order_bin(const SearchArgs& a, uint64_t j, uint32_t lane) {
  const uint32_t nb = __builtin_amdgcn_readfirstlane(a.nbk[j]);
  const uint32_t nj = (uint32_t)(a.off[j + 1] - a.off[j]);
  const float m = (float)max(1u, (uint32_t)(a.toff[j + 1] - a.toff[j]));
  float part = 0.0f;
  for (uint32_t x0 = 0; x0 < nb; x0 += 64) {
    const uint32_t x = x0 + lane;
    const uint32_t k = x < nb ? a.blist[j * a.B + x] >> 16 : 0u;
    if (k >= 8) {
      const float e = min((float)k * (float)(k - 1) / (2.0f * m), 40.0f);
      part += (60.0f + 4.0f * (float)k) * (__expf(e) - 1.0f);
    }
    if (__ballot(k >= 8) != ~0ULL) break;
  }
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) part += __shfl_xor(part, w);
  const float cost = 60.0f * (float)nb + 4.0f * (float)nj + 1.0f + part;
  const int bin = (int)(__log2f(cost) * 16.0f) - 160;
  return __builtin_amdgcn_readfirstlane((uint32_t)min(max(bin, 0), (int)kOrderBins - 1));
}

__global__ void k_order_clear(uint32_t* __restrict__ hist) { hist[threadIdx.x] = 0; }

// One wavefront per partition: its bin to bins[j], counted in the workgroup's LDS histogram, which
// is added to hist with one atomic per non-empty bin.
__global__ __launch_bounds__(kOrderThreads) void k_order_count(SearchArgs a, uint32_t* __restrict__ hist,
                                                               uint8_t* __restrict__ bins) {
  __shared__ uint32_t h[kOrderBins];
  const uint32_t t = threadIdx.x, lane = t & 63;
  constexpr uint32_t kWaves = kOrderThreads / 64;
  if (t < kOrderBins) h[t] = 0;
  __syncthreads();
  for (uint64_t j = (uint64_t)blockIdx.x * kWaves + (t >> 6); j < a.K; j += (uint64_t)gridDim.x * kWaves) {
    const uint32_t b = order_bin(a, j, lane);
    if (lane == 0) {
      bins[j] = (uint8_t)b;
      atomicAdd(&h[b], 1u);
    }
  }
  __syncthreads();
  if (t < kOrderBins && h[t]) atomicAdd(&hist[t], h[t]);
}
// hist[b] -> start of bin b when the bins run from the largest estimate down; cursor cleared
__global__ void k_order_scan(uint32_t* __restrict__ hist, uint32_t* __restrict__ cursor) {
  __shared__ uint32_t v[kOrderBins];
  const uint32_t t = threadIdx.x;
  v[t] = hist[kOrderBins - 1 - t];
  __syncthreads();
  for (uint32_t d = 1; d < kOrderBins; d <<= 1) {
    const uint32_t y = t >= d ? v[t - d] : 0u;
    __syncthreads();
    v[t] += y;
    __syncthreads();
  }
  hist[kOrderBins - 1 - t] = v[t] - hist[kOrderBins - 1 - t];
  cursor[t] = 0;
}

// Workgroup g places the partitions [g kOrderThreads kOrderPer, ...): ranks within the workgroup
// from LDS counts, one global atomic per non-empty bin for the workgroup's range in that bin.
__global__ __launch_bounds__(kOrderThreads) void k_order_scatter(uint64_t K, const uint8_t* __restrict__ bins,
                                                                 const uint32_t* __restrict__ start,
                                                                 uint32_t* __restrict__ cursor,
                                                                 uint32_t* __restrict__ order) {
  __shared__ uint32_t cnt[kOrderBins], base[kOrderBins];
  const uint32_t t = threadIdx.x;
  if (t < kOrderBins) cnt[t] = 0;
  __syncthreads();
  const uint64_t j0 = (uint64_t)blockIdx.x * kOrderThreads * kOrderPer;
  uint32_t b[kOrderPer], r[kOrderPer];
#pragma unroll
  for (uint32_t u = 0; u < kOrderPer; u++) {
    const uint64_t j = j0 + (uint64_t)u * kOrderThreads + t;
    b[u] = j < K ? bins[j] : 0u;
    r[u] = j < K ? atomicAdd(&cnt[b[u]], 1u) : 0u;
  }
  __syncthreads();
  if (t < kOrderBins && cnt[t]) base[t] = start[t] + atomicAdd(&cursor[t], cnt[t]);
  __syncthreads();
#pragma unroll
  for (uint32_t u = 0; u < kOrderPer; u++) {
    const uint64_t j = j0 + (uint64_t)u * kOrderThreads + t;
    if (j < K) order[base[b[u]] + r[u]] = (uint32_t)j;
  }
}

// One wavefront per partition.
template <int kWaves, bool kMulti>
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_search(SearchArgs a) {
  extern __shared__ __align__(16) uint32_t lds32[];
  const uint32_t wave = uniform(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const uint64_t x = (uint64_t)blockIdx.x * kWaves + wave;
  if (x >= a.K) return;
  const uint64_t j = a.order ? (uint64_t)uniform(a.order[x]) : x;
  search_partition<kMulti, false>(a, j, lds32 + (size_t)wave * (a.wave_lds / 4), lane);
}

// Wide partitions: one wavefront per workgroup and partition, with the LDS it needs (up to what one
// workgroup may hold).
__global__ __launch_bounds__(64) void k_search_wide(SearchArgs a) {
  extern __shared__ __align__(16) uint32_t lds32[];
  const uint64_t j = blockIdx.x;
  if (j >= a.K) return;
  search_partition<true, true>(a, j, lds32, threadIdx.x & 63);
}

// Persistent: every wavefront takes `grab` partitions at a time from the queue until none is left.
template <int kWaves, bool kMulti>
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_search_persistent(SearchArgs a) {
  extern __shared__ __align__(16) uint32_t lds32[];
  const uint32_t wave = uniform(threadIdx.x >> 6), lane = threadIdx.x & 63;
  uint32_t* F2 = lds32 + (size_t)wave * (a.wave_lds / 4);
  for (;;) {
    unsigned long long item = 0;
    if (lane == 0) item = atomicAdd(a.queue, (unsigned long long)a.grab);
    item = lane_value64(item, 0);
    if (item >= a.K) break;
    const uint64_t end = min((uint64_t)item + a.grab, a.K);
    for (uint64_t x = item; x < end; x++) {
      const uint64_t j = a.order ? (uint64_t)uniform(a.order[x]) : x;
      search_partition<kMulti, false>(a, j, F2, lane);
      wave_sync();
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Search launch shape
// ---------------------------------------------------------------------------------------------
std::mutex g_cfg_mu;
phobic_search_config g_cfg = {1, 0, 1, 0};  // one partition per workgroup

phobic_search_config search_config() {
  std::lock_guard<std::mutex> lock(g_cfg_mu);
  return g_cfg;
}

template <int W, bool kMulti>
hipError_t launch_search_w(SearchArgs& sa, uint64_t items, const phobic_search_config& cfg, hipStream_t st,
                           unsigned long long* queue) {
  const size_t lds = (size_t)sa.wave_lds * W;
  if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
  if (cfg.groups_per_cu == 0) {
    sa.queue = nullptr;
    hipLaunchKernelGGL((k_search<W, kMulti>), dim3((uint32_t)((items + W - 1) / W)), dim3(64 * W), lds, st, sa);
    return hipGetLastError();
  }
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  sa.queue = queue;
  sa.grab = std::max<uint32_t>(1, cfg.items_per_grab);
  hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, st, queue);
  const uint64_t groups = std::min<uint64_t>((uint64_t)cus * cfg.groups_per_cu, (items + W - 1) / W);
  hipLaunchKernelGGL((k_search_persistent<W, kMulti>), dim3((uint32_t)std::max<uint64_t>(groups, 1)), dim3(64 * W),
                     lds, st, sa);
  return hipGetLastError();
}

// Launches the search over `items` partitions (sa.K) with the configured shape.
}  // namespace

template <bool kMulti>
hipError_t launch_search_m(SearchArgs& sa, uint64_t items, const phobic_search_config& cfg, hipStream_t st,
                           unsigned long long* queue) {
  switch (cfg.waves_per_group) {
    case 1: return launch_search_w<1, kMulti>(sa, items, cfg, st, queue);
    case 2: return launch_search_w<2, kMulti>(sa, items, cfg, st, queue);
    case 8: return launch_search_w<8, kMulti>(sa, items, cfg, st, queue);
    default: return launch_search_w<4, kMulti>(sa, items, cfg, st, queue);
  }
}

hipError_t order_partitions(SearchArgs& sa, uint32_t* order, uint32_t* scratch, hipStream_t st) {
  uint32_t* hist = scratch;
  uint32_t* cursor = scratch + kOrderBins;
  uint8_t* bins = (uint8_t*)(scratch + 2 * kOrderBins);
  const uint32_t cgrid = (uint32_t)std::min<uint64_t>((sa.K + kOrderThreads / 64 - 1) / (kOrderThreads / 64), 1024);
  const uint32_t sgrid = (uint32_t)((sa.K + kOrderThreads * kOrderPer - 1) / (kOrderThreads * kOrderPer));
  sa.order = nullptr;
  hipLaunchKernelGGL(k_order_clear, dim3(1), dim3(kOrderBins), 0, st, hist);
  hipLaunchKernelGGL(k_order_count, dim3(cgrid), dim3(kOrderThreads), 0, st, sa, hist, bins);
  hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(kOrderBins), 0, st, hist, cursor);
  hipLaunchKernelGGL(k_order_scatter, dim3(sgrid), dim3(kOrderThreads), 0, st, sa.K, (const uint8_t*)bins,
                     (const uint32_t*)hist, cursor, order);
  sa.order = order;
  return hipGetLastError();
}

hipError_t launch_search(SearchArgs& sa, uint64_t items, hipStream_t st, unsigned long long* queue) {
  if (sa.wide) {
    sa.queue = nullptr;
    (void)allow_lds(k_search_wide, sa.wave_lds);
    hipLaunchKernelGGL(k_search_wide, dim3((uint32_t)items), dim3(64), sa.wave_lds, st, sa);
    return hipGetLastError();
  }
  const phobic_search_config cfg = search_config();
  // tables of more than 4096 slots need scans of several passes
  return sa.max_m > 4096 ? launch_search_m<true>(sa, items, cfg, st, queue)
                         : launch_search_m<false>(sa, items, cfg, st, queue);
}

}  // namespace phobic

using namespace phobic;

extern "C" phobic_status phobic_set_search_config(const phobic_search_config* cfg) {
  if (!cfg) return fail(PHOBIC_E_INVALID, "cfg is null");
  const uint32_t w = cfg->waves_per_group;
  if (w != 1 && w != 2 && w != 4 && w != 8) return fail(PHOBIC_E_INVALID, "waves_per_group must be 1, 2, 4 or 8");
  if (cfg->groups_per_cu > 64) return fail(PHOBIC_E_INVALID, "groups_per_cu must be at most 64");
  if (cfg->groups_per_cu && (cfg->items_per_grab < 1 || cfg->items_per_grab > 4096))
    return fail(PHOBIC_E_INVALID, "items_per_grab must be in [1, 4096]");
  std::lock_guard<std::mutex> lock(g_cfg_mu);
  g_cfg = *cfg;
  g_cfg.reserved = 0;
  return PHOBIC_OK;
}

extern "C" phobic_status phobic_get_search_config(phobic_search_config* out) {
  if (!out) return fail(PHOBIC_E_INVALID, "out is null");
  *out = search_config();
  return PHOBIC_OK;
}

