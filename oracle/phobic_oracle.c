/*
 * phobic_oracle.c -- reference oracle for PHOBIC construction and query.
 *
 * TEST INFRASTRUCTURE ONLY.  The product library never links, loads or calls this file; only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark do.  It shares no source with the
 * HIP path: the key hash, the bucket table, the search, the codecs and the image layout are written
 * here a second time from their definitions.
 *
 * It renders, plainly and sequentially, the method of "PHOBIC: Perfect Hashing with Optimized Bucket
 * Sizes and Interleaved Coding" (Hermann, Lehmann, Pibiri, Sanders, Walzer; arXiv 2404.18497), in
 * the order the paper gives it:
 *
 *   1. key hashing to a 128-bit master hash code                   (Sec. 5 setup; Sec. 5.1)
 *   2. partitioning into partitions of expected size P             (Sec. 4, first paragraph)
 *   3. bucket assignment by the tabulated function beta_eps        (Sec. 3.1, Sec. 3.2, App. C.1)
 *   4. bucket ordering: size descending, then expected size
 *      ascending                                                   (Sec. 3 intro; Sec. 5.1 "Further remarks")
 *   5. seed (pilot) search with the additive displacement hash     (Sec. 4, "Hash Function")
 *   6. interleaved coding, Compact, Golomb-Rice or a mix of both   (Sec. 4.1)
 *   7. partition offsets stored relative to their expectation       (Sec. 4, "Encoding the offsets")
 *   8. query                                                       (Sec. 4, "Hash Function", last sentences)
 *   9. non-minimal variant with remapping                          (App. B; Sec. 5.1 "Further remarks")
 *
 * Where the paper leaves a detail open, this file follows the readings recorded in the design notes
 * of the repository (hash functions, zero-based buckets, tie order, Rice parameter, select samples,
 * offset expectation, remap layout).  Each such place says so in a comment.
 *
 * Nothing here is blocked, fused or reordered for speed: the search is the nested loop over seeds s,
 * displacements d and keys that Sec. 4 describes.  The only concurrency is an optional split of the
 * independent partitions over threads (Sec. 1, "Partitioning": each partition is built on its own).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ----------------------------------------------------------------------------------------------
 * Status codes (same numbering as the library's, declared independently).
 * -------------------------------------------------------------------------------------------- */
enum {
  REF_OK = 0,
  REF_E_INVALID = 1,
  REF_E_DUPLICATE = 2,
  REF_E_OOM = 3,
  REF_E_PILOT_OVERFLOW = 4,
  REF_E_DEVICE = 5,
  REF_E_FORMAT = 6,
  REF_E_CAPACITY = 7
};

typedef struct {
  uint32_t partition_size; /* P: expected partition size */
  uint32_t coding;         /* 0 = interleaved Golomb-Rice, 1 = interleaved Compact */
  double lambda;           /* average bucket size */
  uint32_t alpha_num;      /* load factor alpha = alpha_num / alpha_den, alpha <= 1 */
  uint32_t alpha_den;
  uint64_t hash_seed;
  uint64_t pilot_limit;    /* largest admissible pilot; 0 means 2^32 - 1 */
  uint32_t n_compact;      /* interleaved Rice: encoders 0 .. n_compact-1 use Compact instead (0..B) */
  uint32_t bucket_fn;      /* bucket assignment function: 0 beta_eps, 1 beta_*, 2 skewed, 3 uniform */
} ref_params;

/* ----------------------------------------------------------------------------------------------
 * 1. Hashing.  The paper computes a master hash code per key with xxHash and notes that this makes
 * construction nearly independent of the key distribution (Sec. 5 setup).  Its exact hash is not
 * part of the method; this project fixes its own 128-bit hash from two published 64-bit
 * finalizers, both bijections of 64-bit words:
 *   mix_a: the SplitMix64 output function (Steele, Lea, Flood 2014; constants of Stafford's
 *          "variant 13"),
 *   mix_b: the MurmurHash3 64-bit finalizer "fmix64" (Appleby).
 * -------------------------------------------------------------------------------------------- */
#define PHI64 0x9E3779B97F4A7C15ULL   /* 2^64 / golden ratio, odd */
#define SQRT2_64 0x6A09E667F3BCC909ULL /* fractional bits of sqrt(2) */

static uint64_t mix_a(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static uint64_t mix_b(uint64_t k) {
  k ^= k >> 33;
  k *= 0xFF51AFD7ED558CCDULL;
  k ^= k >> 33;
  k *= 0xC4CEB9FE1A85EC53ULL;
  k ^= k >> 33;
  return k;
}

static uint64_t mul_hi(uint64_t a, uint64_t b) {
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
}

/* 64-bit key -> (hi, lo).  hi is a bijection of the key, so distinct keys never share hi. */
static void hash_u64(uint64_t key, uint64_t seed, uint64_t *hi, uint64_t *lo) {
  *hi = mix_a(key ^ seed);
  *lo = mix_b(key ^ seed ^ SQRT2_64);
}

/* Byte string -> (hi, lo): two chains over little-endian 8-byte words (the last one zero-padded),
 * each finished with the byte length. */
static void hash_str(const uint8_t *s, uint64_t len, uint64_t seed, uint64_t *hi, uint64_t *lo) {
  uint64_t a = seed, b = seed ^ SQRT2_64;
  for (uint64_t i = 0; i < len; i += 8) {
    uint64_t w = 0;
    for (uint64_t t = 0; t < 8 && i + t < len; t++) w |= (uint64_t)s[i + t] << (8 * t);
    a = mix_a(a ^ w);
    b = mix_b(b ^ w);
  }
  *hi = mix_a(a ^ len);
  *lo = mix_b(b ^ len);
}

/* Seeded position hash h(x, s) in [0, m) (Sec. 4, "Hash Function": the paper needs a hash of the
 * key and the seed s that stays well distributed in small partitions; XOR-ing two fixed hash values
 * without further mixing is what it rules out).  The key enters through its 64-bit fingerprint
 * f = lo ^ mix_b(hi); the seed through the Weyl value (s + 1) * phi; a full mixer follows the XOR. */
static uint64_t fingerprint(uint64_t hi, uint64_t lo) { return lo ^ mix_b(hi); }

static uint64_t pos_hash(uint64_t hi, uint64_t lo, uint64_t s, uint64_t m) {
  uint64_t z = mix_a(fingerprint(hi, lo) ^ ((s + 1) * PHI64));
  return mul_hi(z, m);
}

/* ----------------------------------------------------------------------------------------------
 * 3. Bucket assignment.  beta_*(x) = x + (1 - x) ln(1 - x) (Sec. 3.2), perturbed to
 * beta_eps(x) = eps x + (1 - eps) beta_*(x) (Theorem 2) with eps = lambda / (5 sqrt(P)) (App. C.1).
 * For comparison (Sec. 3.1, the figure of bucket assignment functions) the parameter bucket_fn also
 * selects beta_* itself, the skewed function of PTHash and FCH (the first 60% of the normalized hash
 * range go to the first 30% of the buckets, each part spread evenly: x / 2 below 0.6, then
 * 0.3 + 1.75 (x - 0.6); Sec. 2) and the uniform one of CHD (gamma(x) = x).
 * For a load factor alpha < 1 the function is gamma_alpha(x) = gamma(alpha x) / gamma(alpha)
 * (App. B).  It is tabulated at 2048 equally spaced points and interpolated linearly (App. C.1);
 * the table holds round(2^32 gamma(k / 2048)) for k = 0..2048.
 * -------------------------------------------------------------------------------------------- */
#define TABLE_SIZE 2048

double phobic_ref_beta_star(double x) {
  if (x >= 1.0) return 1.0;
  return x + (1.0 - x) * log1p(-x);
}

double phobic_ref_beta_eps(double x, double eps) {
  return eps * x + (1.0 - eps) * phobic_ref_beta_star(x);
}

double phobic_ref_epsilon(double lambda, uint32_t P) {
  double eps = lambda / (5.0 * sqrt((double)P));
  return eps > 1.0 ? 1.0 : eps;
}

enum { BF_OPTIMIZED = 0, BF_BETA_STAR = 1, BF_SKEW = 2, BF_UNIFORM = 3, BF_COUNT = 4 };

/* The bucket assignment function selected by fn, at x in [0, 1]. */
double phobic_ref_gamma(double x, uint32_t fn, double eps) {
  switch (fn) {
    case BF_BETA_STAR: return phobic_ref_beta_star(x);
    case BF_SKEW: return x <= 0.6 ? 0.5 * x : 0.3 + 1.75 * (x - 0.6);
    case BF_UNIFORM: return x;
    default: return phobic_ref_beta_eps(x, eps);
  }
}

void phobic_ref_bucket_table_fn(double lambda, uint32_t P, uint32_t alpha_num, uint32_t alpha_den, uint32_t fn,
                                uint64_t *T /* TABLE_SIZE + 1 */) {
  double eps = phobic_ref_epsilon(lambda, P);
  double alpha = (double)alpha_num / (double)alpha_den;
  double norm = phobic_ref_gamma(alpha, fn, eps);
  for (int k = 0; k <= TABLE_SIZE; k++) {
    double x = (double)k / TABLE_SIZE;
    double g = (alpha_num == alpha_den) ? phobic_ref_gamma(x, fn, eps)
                                        : phobic_ref_gamma(alpha * x, fn, eps) / norm;
    T[k] = (uint64_t)llround(ldexp(g, 32));
  }
  T[0] = 0;
  T[TABLE_SIZE] = (uint64_t)1 << 32;
}

void phobic_ref_bucket_table(double lambda, uint32_t P, uint32_t alpha_num, uint32_t alpha_den,
                             uint64_t *T /* TABLE_SIZE + 1 */) {
  phobic_ref_bucket_table_fn(lambda, P, alpha_num, alpha_den, BF_OPTIMIZED, T);
}

/* Zero-based bucket of a key: floor(B * gamma~(x)) with x = lo / 2^64 and gamma~ the linear
 * interpolation of the table (the paper's ceil(gamma(x) B) over x in (0, 1], shifted to 0..B-1).
 * The top 11 bits of lo pick the table interval, the next 32 bits are the interpolation weight. */
static uint32_t bucket_of(uint64_t lo, const uint64_t *T, uint32_t B) {
  uint64_t k = lo >> 53;
  uint64_t f = (lo >> 21) & 0xFFFFFFFFULL;
  uint64_t y = T[k] + (((T[k + 1] - T[k]) * f) >> 32);
  uint64_t b = (y * B) >> 32;
  return (uint32_t)(b < B - 1 ? b : B - 1);
}

uint32_t phobic_ref_bucket_of(uint64_t lo, const uint64_t *T, uint32_t B) { return bucket_of(lo, T, B); }

void phobic_ref_buckets(const uint64_t *lo, uint64_t n, const uint64_t *T, uint32_t B, uint32_t *out) {
  for (uint64_t i = 0; i < n; i++) out[i] = bucket_of(lo[i], T, B);
}

/* ----------------------------------------------------------------------------------------------
 * Derived sizes.
 * -------------------------------------------------------------------------------------------- */
static uint64_t num_partitions(uint64_t n, uint32_t P) {
  uint64_t K = (n + P - 1) / P; /* partitions of expected size P (Sec. 4) */
  return K ? K : 1;
}

static uint32_t num_buckets(uint32_t P, double lambda) {
  return (uint32_t)ceil((double)P / lambda); /* B = P / lambda buckets per partition (Sec. 4.1) */
}

/* Table size of a partition with nj keys: nj for alpha = 1, else ceil(nj / alpha) (App. B). */
static uint64_t table_size(uint64_t nj, uint32_t an, uint32_t ad) {
  if (an == ad) return nj;
  return (nj * ad + an - 1) / an;
}

static int validate(const ref_params *p, uint32_t *B) {
  if (!p) return REF_E_INVALID;
  if (p->partition_size < 1 || !(p->lambda > 0.0) || !isfinite(p->lambda)) return REF_E_INVALID;
  if (p->alpha_den == 0 || p->alpha_num == 0 || p->alpha_num > p->alpha_den) return REF_E_INVALID;
  if (p->coding > 1 || p->bucket_fn >= BF_COUNT) return REF_E_INVALID;
  double b = ceil((double)p->partition_size / p->lambda);
  if (b < 1.0 || b > 65535.0) return REF_E_INVALID;
  *B = num_buckets(p->partition_size, p->lambda);
  /* mixed coding (Sec. 4.1: Compact for the large buckets, Rice for the rest) is a variant of the
   * interleaved Rice image; an all-Compact image has no Rice encoders to replace */
  if (p->coding == 0 && p->n_compact > *B) return REF_E_INVALID;
  if (p->coding == 1 && p->n_compact != 0 && p->n_compact != *B) return REF_E_INVALID;
  return REF_OK;
}

/* ----------------------------------------------------------------------------------------------
 * Bit-level helpers for the image (little-endian 64-bit words, bit i of a stream is bit (i mod 64)
 * of word i / 64).
 * -------------------------------------------------------------------------------------------- */
static void put_bits(uint64_t *w, uint64_t pos, uint64_t v, unsigned width) {
  for (unsigned b = 0; b < width; b++)
    if ((v >> b) & 1) w[(pos + b) >> 6] |= (uint64_t)1 << ((pos + b) & 63);
}

static uint64_t get_bits(const uint64_t *w, uint64_t pos, unsigned width) {
  uint64_t v = 0;
  for (unsigned b = 0; b < width; b++)
    if ((w[(pos + b) >> 6] >> ((pos + b) & 63)) & 1) v |= (uint64_t)1 << b;
  return v;
}

static unsigned bit_length(uint64_t v) {
  unsigned b = 0;
  while (v) {
    b++;
    v >>= 1;
  }
  return b;
}

/* Golomb-Rice parameter for a geometric source of mean mu, by the rule of Kiely ("Selecting the
 * Golomb parameter in Rice coding", 2004), which Sec. 4.1 cites:
 *   b = max(0, 1 + floor(log2( ln(phi - 1) / ln(mu / (mu + 1)) ))),   phi the golden ratio. */
uint32_t phobic_ref_rice_param(uint64_t sum, uint64_t count) {
  if (sum == 0 || count == 0) return 0;
  double mu = (double)sum / (double)count;
  double phi = (1.0 + sqrt(5.0)) / 2.0;
  double ratio = log(phi - 1.0) / log(mu / (mu + 1.0));
  double b = 1.0 + floor(log2(ratio));
  if (b < 0.0) b = 0.0;
  if (b > 32.0) b = 32.0;
  return (uint32_t)b;
}

/* ----------------------------------------------------------------------------------------------
 * The image: header words, then sections (each followed by one zero word).
 * -------------------------------------------------------------------------------------------- */
#define MAGIC 0x33304349424F4850ULL /* "PHOBIC03" */
#define HDR_WORDS 24
/* Select samples of the unary stream: one 64-bit entry per SEL_BLOCK ones.  Entry s holds the
 * position of one number SEL_BLOCK*s in its low 32 bits, and for k = 1, 2, 3 the distance from there
 * to one number SEL_BLOCK*s + SEL_SUB*k in the 10-bit field at bit 32 + 10(k-1); SEL_REL_NONE when
 * the distance does not fit (and 0 for ones past the end of the stream). */
#define SEL_BLOCK 256
#define SEL_SUB 64
#define SEL_REL_NONE 1023
enum {
  H_MAGIC = 0, H_N, H_K, H_B, H_P, H_LAMBDA, H_ALPHA, H_CODING, H_SEED, H_TOTAL, H_DMIN, H_WOFF,
  H_SEC_OFF, H_SEC_ENC, H_SEC_DATA, H_SEC_UNARY, H_SEC_SEL, H_SEC_REMAP, H_WREMAP, H_NREMAP,
  H_UBITS, H_WORDS, H_RPART, H_NCOMPACT
};

struct ref_mphf {
  uint64_t n, K;
  uint32_t B;
  ref_params prm;
  uint64_t *words; /* the serialized image */
  uint64_t nwords;
  uint32_t *pilots; /* K x B, partition-major */
  uint64_t *offsets; /* K + 1 table offsets */
  uint64_t counters[4]; /* hash evaluations, slot probes, seeds tried, buckets placed */
};
typedef struct ref_mphf ref_mphf;

/* ----------------------------------------------------------------------------------------------
 * 4 + 5. Per-partition work: bucket the keys, order the buckets, search every pilot.
 * -------------------------------------------------------------------------------------------- */
typedef struct {
  const uint64_t *hi, *lo;  /* keys grouped by partition */
  const uint64_t *kbeg;     /* first key of each partition */
  const uint64_t *toff;     /* table offset of each partition */
  uint64_t K, j0, j1;       /* partitions [j0, j1) belong to this worker */
  uint32_t B;
  const uint64_t *T;
  uint64_t pilot_limit;
  uint32_t *pilots;
  uint8_t *taken_global;    /* T_total flags, for the remap (alpha < 1) */
  int status;
  uint64_t counters[4];
} part_job;

/* Comparison for the processing order: larger size first; among equal sizes the larger bucket
 * index first, i.e. the smaller expected size first (expected size falls with the index). */
typedef struct { uint32_t size, id; } bucket_ref;
static int order_cmp(const void *a, const void *b) {
  const bucket_ref *x = a, *y = b;
  if (x->size != y->size) return x->size > y->size ? -1 : 1;
  if (x->id != y->id) return x->id > y->id ? -1 : 1;
  return 0;
}

static int build_partition(part_job *job, uint64_t j, int dup_only, uint64_t *stamp_buf, uint8_t *taken,
                           uint64_t *r, uint32_t *kb, uint32_t *cnt, uint32_t *start, uint32_t *keyidx,
                           bucket_ref *order) {
  const uint32_t B = job->B;
  uint64_t first = job->kbeg[j], nj = job->kbeg[j + 1] - job->kbeg[j];
  uint64_t m = job->toff[j + 1] - job->toff[j];
  const uint64_t *hi = job->hi + first, *lo = job->lo + first;
  uint32_t *pil = job->pilots + j * B;

  /* bucket of every key, then the keys grouped by bucket (counting sort) */
  memset(cnt, 0, sizeof(uint32_t) * B);
  for (uint64_t i = 0; i < nj; i++) {
    kb[i] = bucket_of(lo[i], job->T, B);
    cnt[kb[i]]++;
  }
  uint32_t acc = 0;
  for (uint32_t b = 0; b < B; b++) {
    start[b] = acc;
    acc += cnt[b];
  }
  for (uint64_t i = 0; i < nj; i++) keyidx[start[kb[i]]++] = (uint32_t)i;
  for (uint32_t b = 0; b < B; b++) start[b] -= cnt[b];

  /* two keys of one bucket with the same fingerprint (in particular, equal keys) get the same
   * position under every seed and can never be separated: report duplicates */
  for (uint32_t b = 0; b < B; b++)
    for (uint32_t x = 0; x < cnt[b]; x++)
      for (uint32_t y = x + 1; y < cnt[b]; y++) {
        uint32_t u = keyidx[start[b] + x], v = keyidx[start[b] + y];
        if (fingerprint(hi[u], lo[u]) == fingerprint(hi[v], lo[v])) return REF_E_DUPLICATE;
      }
  if (dup_only) return REF_OK;

  /* processing order of the non-empty buckets */
  uint32_t nb = 0;
  for (uint32_t b = 0; b < B; b++)
    if (cnt[b]) {
      order[nb].size = cnt[b];
      order[nb].id = b;
      nb++;
    }
  qsort(order, nb, sizeof(bucket_ref), order_cmp);

  /* the search: for every bucket the smallest pilot p = s m + d such that the positions
   * (h(x, s) + d) mod m of its keys are pairwise distinct and not yet taken (Sec. 4).  Seeds s
   * run in the outer loop, displacements d in [0, m) in the middle one, keys in the inner one. */
  memset(taken, 0, m);
  uint64_t stamp = 0;
  for (uint64_t t = 0; t < m; t++) stamp_buf[t] = 0;
  for (uint32_t o = 0; o < nb; o++) {
    uint32_t b = order[o].id, sz = order[o].size;
    const uint32_t *ks = keyidx + start[b];
    int placed = 0;
    for (uint64_t s = 0; !placed; s++) {
      if (s * m > job->pilot_limit) return REF_E_PILOT_OVERFLOW;
      job->counters[2]++;
      for (uint32_t k = 0; k < sz; k++) r[k] = pos_hash(hi[ks[k]], lo[ks[k]], s, m);
      job->counters[0] += sz;
      /* keys of the bucket that collide with each other under s rule out every d */
      stamp++;
      int distinct = 1;
      for (uint32_t k = 0; k < sz && distinct; k++) {
        if (stamp_buf[r[k]] == stamp) distinct = 0;
        stamp_buf[r[k]] = stamp;
      }
      if (!distinct) continue;
      for (uint64_t d = 0; d < m; d++) {
        uint32_t k = 0;
        for (; k < sz; k++) {
          job->counters[1]++;
          uint64_t q = r[k] + d;
          if (q >= m) q -= m;
          if (taken[q]) break;
        }
        if (k == sz) {
          uint64_t p = s * m + d;
          if (p > job->pilot_limit) return REF_E_PILOT_OVERFLOW;
          for (k = 0; k < sz; k++) {
            uint64_t q = r[k] + d;
            if (q >= m) q -= m;
            taken[q] = 1;
          }
          pil[b] = (uint32_t)p;
          placed = 1;
          break;
        }
      }
    }
    job->counters[3]++;
  }
  if (job->taken_global) memcpy(job->taken_global + job->toff[j], taken, m);
  return REF_OK;
}

static void *part_worker(void *arg) {
  part_job *job = arg;
  uint64_t maxn = 0, maxm = 0;
  for (uint64_t j = job->j0; j < job->j1; j++) {
    uint64_t nj = job->kbeg[j + 1] - job->kbeg[j], m = job->toff[j + 1] - job->toff[j];
    if (nj > maxn) maxn = nj;
    if (m > maxm) maxm = m;
  }
  uint64_t *stamp = malloc(sizeof(uint64_t) * (maxm + 1));
  uint8_t *taken = malloc(maxm + 1);
  uint64_t *r = malloc(sizeof(uint64_t) * (maxn + 1));
  uint32_t *kb = malloc(sizeof(uint32_t) * (maxn + 1));
  uint32_t *keyidx = malloc(sizeof(uint32_t) * (maxn + 1));
  uint32_t *cnt = malloc(sizeof(uint32_t) * job->B);
  uint32_t *start = malloc(sizeof(uint32_t) * job->B);
  bucket_ref *order = malloc(sizeof(bucket_ref) * job->B);
  if (!stamp || !taken || !r || !kb || !keyidx || !cnt || !start || !order) {
    job->status = REF_E_OOM;
  } else {
    /* equal codes anywhere are reported as duplicates, before any search */
    for (uint64_t j = job->j0; j < job->j1 && job->status == REF_OK; j++)
      job->status = build_partition(job, j, 1, stamp, taken, r, kb, cnt, start, keyidx, order);
    for (uint64_t j = job->j0; j < job->j1 && job->status == REF_OK; j++)
      job->status = build_partition(job, j, 0, stamp, taken, r, kb, cnt, start, keyidx, order);
  }
  free(stamp); free(taken); free(r); free(kb); free(keyidx); free(cnt); free(start); free(order);
  return NULL;
}

/* Steps 3-5 for one partition given its codes and table size m: pilots[0..B) of that partition. */
int phobic_ref_search_partition(const uint64_t *hi, const uint64_t *lo, uint64_t nj, uint64_t m,
                                const ref_params *prm, uint32_t *pilots, uint64_t *counters) {
  uint32_t B;
  int st = validate(prm, &B);
  if (st) return st;
  if (m < nj) return REF_E_INVALID;
  uint64_t T[TABLE_SIZE + 1];
  phobic_ref_bucket_table_fn(prm->lambda, prm->partition_size, prm->alpha_num, prm->alpha_den, prm->bucket_fn, T);
  uint64_t kbeg[2] = {0, nj}, toff[2] = {0, m};
  part_job job;
  memset(&job, 0, sizeof(job));
  job.hi = hi; job.lo = lo; job.kbeg = kbeg; job.toff = toff; job.K = 1; job.j0 = 0; job.j1 = 1;
  job.B = B; job.T = T; job.pilot_limit = prm->pilot_limit ? prm->pilot_limit : 0xFFFFFFFFULL;
  job.pilots = pilots; job.status = REF_OK;
  memset(pilots, 0, sizeof(uint32_t) * B);
  part_worker(&job);
  if (counters) memcpy(counters, job.counters, sizeof(job.counters));
  return job.status;
}

/* ----------------------------------------------------------------------------------------------
 * 6 + 7. Encoding into the image.
 * -------------------------------------------------------------------------------------------- */
/* Expected table offset of partition j: floor(j * R / 2^32) with R = floor(T_total 2^32 / K). */
static uint64_t expected_offset(uint64_t j, uint64_t R) {
  return (uint64_t)(((unsigned __int128)j * R) >> 32);
}

static int encode(ref_mphf *h, const uint8_t *taken_global) {
  const uint64_t K = h->K, n = h->n;
  const uint32_t B = h->B;
  const uint64_t Ttot = h->offsets[K];
  const int rice = h->prm.coding == 0;
  /* mixed interleaved coding: encoder i is Compact for i < c and Golomb-Rice for i >= c (the first
   * buckets are the largest, hence queried most often; Sec. 4.1) */
  const uint32_t c = rice ? h->prm.n_compact : 0;

  /* partition offsets as differences to their expectation, shifted by the minimum (Sec. 4) */
  uint64_t R = (uint64_t)(((unsigned __int128)Ttot << 32) / K);
  int64_t dmin = 0;
  for (uint64_t j = 0; j <= K; j++) {
    int64_t dj = (int64_t)(h->offsets[j] - expected_offset(j, R));
    if (j == 0 || dj < dmin) dmin = dj;
  }
  uint64_t umax = 0;
  for (uint64_t j = 0; j <= K; j++) {
    uint64_t u = (uint64_t)((int64_t)(h->offsets[j] - expected_offset(j, R)) - dmin);
    if (u > umax) umax = u;
  }
  unsigned woff = bit_length(umax);

  /* per-encoder parameter: encoder i holds the pilots of bucket i of all K partitions (Sec. 4.1);
   * Compact takes the bit length of the largest value, Rice Kiely's parameter */
  uint32_t *width = calloc(B, sizeof(uint32_t));
  uint64_t *base = calloc(B, sizeof(uint64_t));
  if (!width || !base) { free(width); free(base); return REF_E_OOM; }
  uint64_t data_bits = 0, unary_bits = 0;
  for (uint32_t i = 0; i < B; i++) {
    uint64_t sum = 0, mx = 0;
    for (uint64_t j = 0; j < K; j++) {
      uint64_t v = h->pilots[j * B + i];
      sum += v;
      if (v > mx) mx = v;
    }
    const int enc_rice = rice && i >= c;
    width[i] = enc_rice ? phobic_ref_rice_param(sum, K) : bit_length(mx);
    base[i] = data_bits;
    data_bits += (uint64_t)width[i] * K;
    if (enc_rice)
      for (uint64_t j = 0; j < K; j++) unary_bits += ((uint64_t)h->pilots[j * B + i] >> width[i]) + 1;
  }
  if (rice && unary_bits > 0xFFFFFFFFULL) { free(width); free(base); return REF_E_CAPACITY; }

  /* the remap for alpha < 1: table positions >= n that hold a key, ascending, are paired with the
   * free positions < n, ascending; entries of free positions >= n repeat the previous value */
  uint64_t nremap = Ttot - n;
  unsigned wremap = n > 1 ? bit_length(n - 1) : 0;

  uint64_t sec_off = HDR_WORDS;
  uint64_t sec_enc = sec_off + ((K + 1) * woff + 63) / 64 + 1;
  uint64_t sec_data = sec_enc + B + 1;
  uint64_t sec_unary = sec_data + (data_bits + 63) / 64 + 1;
  uint64_t nvals = K * (B - c); /* values of the Rice encoders, each one a one of the unary stream */
  uint64_t nsel = rice ? (nvals + SEL_BLOCK - 1) / SEL_BLOCK : 0;
  uint64_t sec_sel = sec_unary + (rice ? (unary_bits + 63) / 64 + 1 : 0);
  uint64_t sec_remap = sec_sel + (rice ? nsel + 1 : 0);
  uint64_t total = sec_remap + (nremap ? (nremap * wremap + 63) / 64 + 1 : 0);

  uint64_t *w = calloc(total, sizeof(uint64_t));
  if (!w) { free(width); free(base); return REF_E_OOM; }
  w[H_MAGIC] = MAGIC;
  w[H_N] = n;
  w[H_K] = K;
  w[H_B] = B;
  w[H_P] = h->prm.partition_size;
  memcpy(&w[H_LAMBDA], &h->prm.lambda, 8);
  w[H_ALPHA] = (uint64_t)h->prm.alpha_num | ((uint64_t)h->prm.alpha_den << 32);
  w[H_CODING] = h->prm.coding | ((uint64_t)h->prm.bucket_fn << 8); /* coding, bucket function */
  w[H_SEED] = h->prm.hash_seed;
  w[H_TOTAL] = Ttot;
  w[H_DMIN] = (uint64_t)dmin;
  w[H_WOFF] = woff;
  w[H_SEC_OFF] = sec_off;
  w[H_SEC_ENC] = sec_enc;
  w[H_SEC_DATA] = sec_data;
  w[H_SEC_UNARY] = sec_unary;
  w[H_SEC_SEL] = sec_sel;
  w[H_SEC_REMAP] = sec_remap;
  w[H_WREMAP] = wremap;
  w[H_NREMAP] = nremap;
  w[H_UBITS] = rice ? unary_bits : 0;
  w[H_WORDS] = total;
  w[H_RPART] = R;
  w[H_NCOMPACT] = c;

  for (uint64_t j = 0; j <= K; j++) {
    uint64_t u = (uint64_t)((int64_t)(h->offsets[j] - expected_offset(j, R)) - dmin);
    put_bits(w + sec_off, j * woff, u, woff);
  }
  for (uint32_t i = 0; i < B; i++) w[sec_enc + i] = (base[i] << 8) | width[i];

  /* Compact: fixed width per encoder.  Golomb-Rice: the low width[i] bits compact, the rest as
   * q = v >> width[i] in unary (q zeros then a one) in one stream ordered encoder by encoder; the
   * stream holds the Rice encoders only, so value j of encoder i >= c is its one number (i - c) K + j. */
  uint64_t upos = 0, ones = 0;
  for (uint32_t i = 0; i < B; i++)
    for (uint64_t j = 0; j < K; j++) {
      uint64_t v = h->pilots[j * B + i];
      unsigned wd = width[i];
      uint64_t low = wd >= 64 ? v : (v & (((uint64_t)1 << wd) - 1));
      put_bits(w + sec_data, base[i] + j * wd, low, wd);
      if (rice && i >= c) {
        upos += v >> wd;
        w[sec_unary + (upos >> 6)] |= (uint64_t)1 << (upos & 63);
        if (ones % SEL_SUB == 0) {
          uint64_t *e = &w[sec_sel + ones / SEL_BLOCK];
          unsigned k = (unsigned)(ones % SEL_BLOCK / SEL_SUB);
          if (k == 0) {
            *e = upos & 0xFFFFFFFFULL;
          } else {
            uint64_t rel = upos - (*e & 0xFFFFFFFFULL);
            *e |= (rel < SEL_REL_NONE ? rel : SEL_REL_NONE) << (32 + 10 * (k - 1));
          }
        }
        ones++;
        upos++;
      }
    }

  if (nremap) {
    uint64_t freep = 0; /* next free position < n */
    uint64_t prev = 0;
    for (uint64_t g = n; g < Ttot; g++) {
      uint64_t val = prev;
      if (taken_global[g]) {
        while (taken_global[freep]) freep++;
        val = freep++;
      }
      put_bits(w + sec_remap, (g - n) * wremap, val, wremap);
      prev = val;
    }
  }
  free(width);
  free(base);
  h->words = w;
  h->nwords = total;
  return REF_OK;
}

/* ----------------------------------------------------------------------------------------------
 * Build: steps 1-7 above.
 * -------------------------------------------------------------------------------------------- */
static int build_from_hashes(uint64_t *hi, uint64_t *lo, uint64_t n, const ref_params *prm,
                             int threads, ref_mphf **out) {
  uint32_t B;
  int st = validate(prm, &B);
  if (st) return st;
  ref_mphf *h = calloc(1, sizeof(ref_mphf));
  if (!h) return REF_E_OOM;
  h->n = n;
  h->prm = *prm;
  h->B = B;
  uint64_t K = num_partitions(n, prm->partition_size);
  h->K = K;
  uint64_t limit = prm->pilot_limit ? prm->pilot_limit : 0xFFFFFFFFULL;

  uint64_t T[TABLE_SIZE + 1];
  phobic_ref_bucket_table_fn(prm->lambda, prm->partition_size, prm->alpha_num, prm->alpha_den, prm->bucket_fn, T);

  /* 2. partition j = floor(hi K / 2^64); group the keys by partition */
  uint64_t *kbeg = calloc(K + 1, sizeof(uint64_t));
  uint64_t *toff = calloc(K + 1, sizeof(uint64_t));
  uint64_t *ghi = malloc(sizeof(uint64_t) * (n + 1)), *glo = malloc(sizeof(uint64_t) * (n + 1));
  h->pilots = calloc(K * B, sizeof(uint32_t));
  h->offsets = toff;
  if (!kbeg || !toff || !ghi || !glo || !h->pilots) { st = REF_E_OOM; goto fail; }
  for (uint64_t i = 0; i < n; i++) kbeg[mul_hi(hi[i], K) + 1]++;
  for (uint64_t j = 0; j < K; j++) kbeg[j + 1] += kbeg[j];
  for (uint64_t j = 0; j < K; j++)
    toff[j + 1] = toff[j] + table_size(kbeg[j + 1] - kbeg[j], prm->alpha_num, prm->alpha_den);
  {
    uint64_t *fill = malloc(sizeof(uint64_t) * K);
    if (!fill) { st = REF_E_OOM; goto fail; }
    memcpy(fill, kbeg, sizeof(uint64_t) * K);
    for (uint64_t i = 0; i < n; i++) {
      uint64_t j = mul_hi(hi[i], K);
      ghi[fill[j]] = hi[i];
      glo[fill[j]] = lo[i];
      fill[j]++;
    }
    free(fill);
  }

  uint8_t *taken_global = NULL;
  if (toff[K] > n) {
    taken_global = calloc(toff[K], 1);
    if (!taken_global) { st = REF_E_OOM; goto fail; }
  }

  /* 3-5 per partition, partitions split over threads */
  if (threads < 1) threads = 1;
  if ((uint64_t)threads > K) threads = (int)K;
  part_job *jobs = calloc(threads, sizeof(part_job));
  pthread_t *tid = calloc(threads, sizeof(pthread_t));
  if (!jobs || !tid) { free(jobs); free(tid); free(taken_global); st = REF_E_OOM; goto fail; }
  for (int t = 0; t < threads; t++) {
    part_job *jb = &jobs[t];
    jb->hi = ghi; jb->lo = glo; jb->kbeg = kbeg; jb->toff = toff; jb->K = K; jb->B = B; jb->T = T;
    jb->j0 = K * t / threads; jb->j1 = K * (t + 1) / threads;
    jb->pilot_limit = limit; jb->pilots = h->pilots; jb->taken_global = taken_global;
    jb->status = REF_OK;
  }
  if (threads == 1) {
    part_worker(&jobs[0]);
  } else {
    for (int t = 0; t < threads; t++) pthread_create(&tid[t], NULL, part_worker, &jobs[t]);
    for (int t = 0; t < threads; t++) pthread_join(tid[t], NULL);
  }
  st = REF_OK;
  for (int t = 0; t < threads; t++) {
    /* report the error of the lowest partition range; duplicates take precedence over overflow */
    if (jobs[t].status == REF_E_DUPLICATE) { st = REF_E_DUPLICATE; break; }
    if (jobs[t].status && !st) st = jobs[t].status;
  }
  for (int t = 0; t < threads; t++)
    for (int c = 0; c < 4; c++) h->counters[c] += jobs[t].counters[c];
  free(jobs);
  free(tid);
  if (st) { free(taken_global); goto fail; }

  st = encode(h, taken_global);
  free(taken_global);
  if (st) goto fail;
  free(kbeg); free(ghi); free(glo);
  *out = h;
  return REF_OK;

fail:
  free(kbeg); free(ghi); free(glo);
  free(h->pilots); free(h->offsets); free(h->words); free(h);
  *out = NULL;
  return st;
}

/* ----------------------------------------------------------------------------------------------
 * 8. Query, reading only the image.
 * -------------------------------------------------------------------------------------------- */
static uint64_t select_one(const uint64_t *unary, const uint64_t *sel, uint64_t t) {
  /* position of the t-th one (t counted from 0) of the unary stream: from the nearest sample at or
   * before it, then one bit at a time */
  uint64_t e = sel[t / SEL_BLOCK];
  uint64_t pos = e & 0xFFFFFFFFULL;
  uint64_t left = t % SEL_BLOCK;
  unsigned k = (unsigned)(left / SEL_SUB);
  uint64_t rel = k ? (e >> (32 + 10 * (k - 1))) & 1023 : SEL_REL_NONE;
  if (rel != SEL_REL_NONE) {
    pos += rel;
    left %= SEL_SUB;
  }
  for (;;) {
    if ((unary[pos >> 6] >> (pos & 63)) & 1) {
      if (left == 0) return pos;
      left--;
    }
    pos++;
  }
}

static void image_table(const uint64_t *w, uint64_t *T) {
  double lambda;
  memcpy(&lambda, &w[H_LAMBDA], 8);
  phobic_ref_bucket_table_fn(lambda, (uint32_t)w[H_P], (uint32_t)w[H_ALPHA], (uint32_t)(w[H_ALPHA] >> 32),
                             (uint32_t)(w[H_CODING] >> 8), T);
}

static uint64_t query_hash(const uint64_t *w, const uint64_t *T, uint64_t hi, uint64_t lo) {
  const uint64_t n = w[H_N], K = w[H_K];
  const uint32_t B = (uint32_t)w[H_B];
  const uint64_t R = w[H_RPART];
  const int64_t dmin = (int64_t)w[H_DMIN];
  const unsigned woff = (unsigned)w[H_WOFF];
  const uint64_t *off = w + w[H_SEC_OFF];
  if (n == 0) return 0;

  uint64_t j = mul_hi(hi, K);
  uint64_t o0 = expected_offset(j, R) + (uint64_t)dmin + get_bits(off, j * woff, woff);
  uint64_t o1 = expected_offset(j + 1, R) + (uint64_t)dmin + get_bits(off, (j + 1) * woff, woff);
  uint64_t m = o1 - o0;
  if (m == 0) return o0 < n ? o0 : n - 1; /* only a non-member can land in an empty partition */

  uint32_t i = bucket_of(lo, T, B);

  uint64_t e = w[w[H_SEC_ENC] + i];
  unsigned wd = (unsigned)(e & 0xFF);
  uint64_t p = get_bits(w + w[H_SEC_DATA], (e >> 8) + j * wd, wd);
  const uint64_t c = w[H_NCOMPACT]; /* encoders below c are Compact */
  if ((w[H_CODING] & 0xFF) == 0 && i >= c) {
    uint64_t t = (uint64_t)(i - c) * K + j;
    const uint64_t *un = w + w[H_SEC_UNARY], *sel = w + w[H_SEC_SEL];
    uint64_t pt = select_one(un, sel, t);
    uint64_t prev = t ? select_one(un, sel, t - 1) : (uint64_t)-1;
    uint64_t q = pt - prev - 1;
    p |= q << wd;
  }
  /* position (h(x, floor(p / m)) + p) mod m (Sec. 4, "Hash Function") */
  uint64_t pos = (pos_hash(hi, lo, p / m, m) + p) % m;
  uint64_t g = o0 + pos;
  if (g < n) return g;
  return get_bits(w + w[H_SEC_REMAP], (g - n) * w[H_WREMAP], (unsigned)w[H_WREMAP]);
}

/* ----------------------------------------------------------------------------------------------
 * Exported entry points (ctypes).
 * -------------------------------------------------------------------------------------------- */
void phobic_ref_hash_u64(const uint64_t *keys, uint64_t n, uint64_t seed, uint64_t *hi, uint64_t *lo) {
  for (uint64_t i = 0; i < n; i++) hash_u64(keys[i], seed, &hi[i], &lo[i]);
}

void phobic_ref_hash_str(const uint8_t *bytes, const uint64_t *offs, uint64_t n, uint64_t seed,
                         uint64_t *hi, uint64_t *lo) {
  for (uint64_t i = 0; i < n; i++) hash_str(bytes + offs[i], offs[i + 1] - offs[i], seed, &hi[i], &lo[i]);
}

uint64_t phobic_ref_pos_hash(uint64_t hi, uint64_t lo, uint64_t s, uint64_t m) { return pos_hash(hi, lo, s, m); }
uint64_t phobic_ref_mix_a(uint64_t z) { return mix_a(z); }
uint64_t phobic_ref_mix_b(uint64_t z) { return mix_b(z); }

uint64_t phobic_ref_partition_of(uint64_t hi, uint64_t K) { return mul_hi(hi, K); }

int phobic_ref_build_hashes(const uint64_t *hi, const uint64_t *lo, uint64_t n, const ref_params *prm,
                            int threads, ref_mphf **out) {
  uint64_t *a = malloc(sizeof(uint64_t) * (n + 1)), *b = malloc(sizeof(uint64_t) * (n + 1));
  if (!a || !b) { free(a); free(b); return REF_E_OOM; }
  memcpy(a, hi, sizeof(uint64_t) * n);
  memcpy(b, lo, sizeof(uint64_t) * n);
  int st = build_from_hashes(a, b, n, prm, threads, out);
  free(a);
  free(b);
  return st;
}

int phobic_ref_build_u64(const uint64_t *keys, uint64_t n, const ref_params *prm, int threads, ref_mphf **out) {
  *out = NULL;
  if (!prm) return REF_E_INVALID;
  uint64_t *a = malloc(sizeof(uint64_t) * (n + 1)), *b = malloc(sizeof(uint64_t) * (n + 1));
  if (!a || !b) { free(a); free(b); return REF_E_OOM; }
  phobic_ref_hash_u64(keys, n, prm->hash_seed, a, b);
  int st = build_from_hashes(a, b, n, prm, threads, out);
  free(a);
  free(b);
  return st;
}

int phobic_ref_build_str(const uint8_t *bytes, const uint64_t *offs, uint64_t n, const ref_params *prm,
                         int threads, ref_mphf **out) {
  *out = NULL;
  if (!prm) return REF_E_INVALID;
  uint64_t *a = malloc(sizeof(uint64_t) * (n + 1)), *b = malloc(sizeof(uint64_t) * (n + 1));
  if (!a || !b) { free(a); free(b); return REF_E_OOM; }
  phobic_ref_hash_str(bytes, offs, n, prm->hash_seed, a, b);
  int st = build_from_hashes(a, b, n, prm, threads, out);
  free(a);
  free(b);
  return st;
}

void phobic_ref_query_u64(const ref_mphf *h, const uint64_t *keys, uint64_t n, uint64_t *out) {
  uint64_t T[TABLE_SIZE + 1];
  image_table(h->words, T);
  for (uint64_t i = 0; i < n; i++) {
    uint64_t hi, lo;
    hash_u64(keys[i], h->prm.hash_seed, &hi, &lo);
    out[i] = query_hash(h->words, T, hi, lo);
  }
}

void phobic_ref_query_str(const ref_mphf *h, const uint8_t *bytes, const uint64_t *offs, uint64_t n,
                          uint64_t *out) {
  uint64_t T[TABLE_SIZE + 1];
  image_table(h->words, T);
  for (uint64_t i = 0; i < n; i++) {
    uint64_t hi, lo;
    hash_str(bytes + offs[i], offs[i + 1] - offs[i], h->prm.hash_seed, &hi, &lo);
    out[i] = query_hash(h->words, T, hi, lo);
  }
}

/* query straight from an image (e.g. one the GPU library serialized), byte-string keys */
int phobic_ref_query_image_str(const uint64_t *words, uint64_t nwords, const uint8_t *bytes, const uint64_t *offs,
                               uint64_t n, uint64_t *out) {
  if (nwords < HDR_WORDS || words[H_MAGIC] != MAGIC || words[H_WORDS] != nwords) return REF_E_FORMAT;
  uint64_t T[TABLE_SIZE + 1];
  image_table(words, T);
  for (uint64_t i = 0; i < n; i++) {
    uint64_t hi, lo;
    hash_str(bytes + offs[i], offs[i + 1] - offs[i], words[H_SEED], &hi, &lo);
    out[i] = query_hash(words, T, hi, lo);
  }
  return REF_OK;
}

/* query straight from an image (e.g. one the GPU library serialized) */
int phobic_ref_query_image_u64(const uint64_t *words, uint64_t nwords, const uint64_t *keys, uint64_t n,
                               uint64_t *out) {
  if (nwords < HDR_WORDS || words[H_MAGIC] != MAGIC || words[H_WORDS] != nwords) return REF_E_FORMAT;
  uint64_t T[TABLE_SIZE + 1];
  image_table(words, T);
  for (uint64_t i = 0; i < n; i++) {
    uint64_t hi, lo;
    hash_u64(keys[i], words[H_SEED], &hi, &lo);
    out[i] = query_hash(words, T, hi, lo);
  }
  return REF_OK;
}

uint64_t phobic_ref_num_words(const ref_mphf *h) { return h->nwords; }
const uint64_t *phobic_ref_words(const ref_mphf *h) { return h->words; }
uint64_t phobic_ref_num_partitions(const ref_mphf *h) { return h->K; }
uint32_t phobic_ref_num_buckets(const ref_mphf *h) { return h->B; }
void phobic_ref_get_pilots(const ref_mphf *h, uint32_t *out) { memcpy(out, h->pilots, sizeof(uint32_t) * h->K * h->B); }
void phobic_ref_get_offsets(const ref_mphf *h, uint64_t *out) { memcpy(out, h->offsets, sizeof(uint64_t) * (h->K + 1)); }
void phobic_ref_get_counters(const ref_mphf *h, uint64_t *out) { memcpy(out, h->counters, sizeof(h->counters)); }
uint64_t phobic_ref_num_partitions_for(uint64_t n, uint32_t P) { return num_partitions(n, P); }
uint32_t phobic_ref_num_buckets_for(uint32_t P, double lambda) { return num_buckets(P, lambda); }

void phobic_ref_free(ref_mphf *h) {
  if (!h) return;
  free(h->words);
  free(h->pilots);
  free(h->offsets);
  free(h);
}
