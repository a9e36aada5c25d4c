/*
 * phobic.h -- C ABI of the MI355X PHOBIC library (libphobic.so).
 *
 * PHOBIC (Hermann, Lehmann, Pibiri, Sanders, Walzer: "PHOBIC: Perfect Hashing with Optimized Bucket
 * Sizes and Interleaved Coding", arXiv 2404.18497) builds a minimal perfect hash function: a
 * bijection from a key set S onto [0, n), n = |S|, that may map keys outside S anywhere (Sec. 1).
 *
 * Conventions for every entry point:
 *  - Pointers named d_* are device pointers (HBM of the current HIP device); h_* are host pointers.
 *    The caller owns all of them; the library never frees or retains them past the call.
 *  - `hip_stream` is a hipStream_t (NULL = the default stream). All device work of a call is
 *    enqueued on it.
 *  - The library owns every phobic_mphf and its device memory until phobic_free().  A handle is
 *    immutable after it is returned, so concurrent queries on one handle are safe.
 *  - No exception crosses the ABI.  On failure a call returns a status other than PHOBIC_OK, sets
 *    *out to NULL where it has one, frees what it allocated, and leaves a message for
 *    phobic_last_error() (per thread).
 *  - The device that is current when a handle is built or deserialized is the handle's device;
 *    queries must run with that device current.
 */
#ifndef PHOBIC_H
#define PHOBIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PHOBIC_OK = 0,
  PHOBIC_E_INVALID = 1,        /* bad argument or parameter */
  PHOBIC_E_DUPLICATE = 2,      /* two keys of one bucket share their 64-bit fingerprint (equal keys) */
  PHOBIC_E_OOM = 3,            /* device or host allocation failed */
  PHOBIC_E_PILOT_OVERFLOW = 4, /* a bucket needs a pilot above params.pilot_limit */
  PHOBIC_E_DEVICE = 5,         /* a HIP runtime call failed */
  PHOBIC_E_FORMAT = 6,         /* a serialized image is malformed */
  PHOBIC_E_CAPACITY = 7        /* a partition or bucket exceeds what one workgroup holds in LDS */
} phobic_status;

enum { PHOBIC_IC_RICE = 0, PHOBIC_IC_COMPACT = 1 };
/* Bucket assignment functions (Sec. 3.1, Sec. 3.2): PHOBIC's beta_eps (the default), beta_* itself,
 * and for comparison the skewed function of PTHash and FCH (60% of the hash range onto the first 30%
 * of the buckets) and the uniform one of CHD. */
enum { PHOBIC_BF_OPTIMIZED = 0, PHOBIC_BF_BETA_STAR = 1, PHOBIC_BF_SKEW = 2, PHOBIC_BF_UNIFORM = 3 };
enum { PHOBIC_FLAG_KEEP_PILOTS = 1u }; /* keep the raw pilot array for phobic_get_pilots() */

/* Construction parameters (Sec. 4, Sec. 4.1, Sec. 5; App. B for alpha). */
typedef struct {
  uint32_t partition_size; /* P: expected keys per partition; default 2500 (Sec. 5 setup) */
  uint32_t coding;         /* PHOBIC_IC_RICE (interleaved Golomb-Rice) or PHOBIC_IC_COMPACT */
  double lambda;           /* average bucket size; B = ceil(P / lambda) buckets per partition */
  uint32_t alpha_num;      /* load factor alpha = alpha_num / alpha_den in (0, 1]; 1/1 = minimal; */
  uint32_t alpha_den;      /*   alpha < 1 builds a table of ceil(n_j / alpha) slots and remaps */
  uint64_t hash_seed;      /* seed of the 128-bit key hash */
  uint64_t pilot_limit;    /* largest admissible pilot; 0 = 2^32 - 1 */
  uint32_t n_compact;      /* mixed interleaved coding (Sec. 4.1): with PHOBIC_IC_RICE, encoders
                              0 .. n_compact-1 (the largest, most queried buckets) use Compact and the
                              rest Golomb-Rice; 0 .. B.  With PHOBIC_IC_COMPACT it must be 0 or B. */
  uint32_t flags;          /* PHOBIC_FLAG_* */
  uint32_t bucket_function; /* PHOBIC_BF_*; stored in the image (bits 8.. of the coding word) */
  uint32_t reserved;        /* must be 0 */
} phobic_params;

typedef struct phobic_mphf phobic_mphf;

/* Per-phase device times of one build, in milliseconds, from HIP events on the build stream. */
typedef struct {
  double hash_count_ms;  /* hash + partition histogram */
  double scan_ms;        /* partition offsets */
  double scatter_ms;     /* hash + scatter into partitions */
  double bucket_sort_ms; /* bucket mapping and ordering */
  double search_ms;      /* pilot search */
  double encode_ms;      /* statistics, packing, remap */
  double total_ms;       /* first kernel to last, host round trips included */
  uint64_t max_partition_keys;
  uint32_t max_bucket_keys;
  uint32_t partition_path; /* 0: coarse bins of a few partitions, two splits and a per-bin sort;
                              1: the general path (per-key global atomics), taken when the coarse
                              bins would not fit one histogram or n >= 2^32 */
} phobic_build_info;

/* Fills *p with the defaults: P = 2500, lambda = 7, alpha = 1, interleaved Rice, seed 0x5EED. */
void phobic_params_default(phobic_params* p);

/* Builds the MPHF of the n distinct 64-bit keys d_keys[0..n) (device, 8-byte aligned).
 * Steps: hash, partition, bucket by beta_eps, order, pilot search, interleaved coding (Sec. 3,
 * Sec. 4, Sec. 4.1, Sec. 4.2).  Returns when the work on hip_stream is complete.  n = 0 gives a
 * valid empty handle.  Equal keys give PHOBIC_E_DUPLICATE. */
phobic_status phobic_build_u64(const uint64_t* d_keys, uint64_t n, const phobic_params* params,
                               void* hip_stream, phobic_mphf** out);

/* As phobic_build_u64 for n byte strings: string i is d_bytes[d_offsets[i] .. d_offsets[i+1]);
 * d_offsets has n + 1 entries (device, non-decreasing). */
phobic_status phobic_build_str(const uint8_t* d_bytes, const uint64_t* d_offsets, uint64_t n,
                               const phobic_params* params, void* hip_stream, phobic_mphf** out);

/* Evaluates the MPHF for n keys: d_pos[i] = position of d_keys[i] (Sec. 4, "Hash Function":
 * (h(x, floor(p / m)) + p) mod m plus the partition offset).  Keys of the build set get distinct
 * positions in [0, n); other keys get an arbitrary position in [0, n).  Asynchronous on
 * hip_stream. */
phobic_status phobic_query_u64(const phobic_mphf* h, const uint64_t* d_keys, uint64_t n, uint64_t* d_pos,
                               void* hip_stream);

/* As phobic_query_u64 for byte strings laid out as in phobic_build_str. */
phobic_status phobic_query_str(const phobic_mphf* h, const uint8_t* d_bytes, const uint64_t* d_offsets,
                               uint64_t n, uint64_t* d_pos, void* hip_stream);

/* Evaluates `count` requests in one launch: request r queries h_handles[r] for the h_counts[r] keys
 * at the device pointer h_keys[r] and writes positions to the device pointer h_outs[r] (all four are
 * host arrays of `count` entries; handles may differ and must live on the current device).  Every
 * output equals that of a separate phobic_query_u64.  Asynchronous on hip_stream; the host arrays
 * may be reused as soon as the call returns. */
phobic_status phobic_query_multi_u64(const phobic_mphf* const* h_handles, const uint64_t* const* h_keys,
                                     const uint64_t* h_counts, uint64_t* const* h_outs, uint32_t count,
                                     void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): phobic_query_multi_u64 without any allocation.  Same arguments
 * and outputs; the per-call job table goes to a fixed device array of the library (one per GPU, about
 * 0.7 MB, held until the process ends) instead of the library's memory pool.  At most
 * PHOBIC_NOALLOC_MAX_REQUESTS requests per call (more give PHOBIC_E_INVALID and no work).  Every call
 * on one GPU shares that GPU's array, so calls must not overlap on a GPU: issue them on one stream,
 * or order them (events, synchronization); overlapping calls race on the table.  Asynchronous on
 * hip_stream like phobic_query_multi_u64. */
#define PHOBIC_NOALLOC_MAX_REQUESTS 4096
phobic_status phobic_query_multi_u64_noalloc(const phobic_mphf* const* h_handles, const uint64_t* const* h_keys,
                                             const uint64_t* h_counts, uint64_t* const* h_outs, uint32_t count,
                                             void* hip_stream);

/* Size of the structure in bits = 8 x serialized bytes, header and tables included; divided by n it
 * is the space measure (bits per key) of Sec. 5 and Table 1. */
uint64_t phobic_size_bits(const phobic_mphf* h);
uint64_t phobic_num_keys(const phobic_mphf* h);
uint64_t phobic_num_partitions(const phobic_mphf* h);
uint32_t phobic_num_buckets(const phobic_mphf* h);

/* Copies the pilots (the per-bucket seeds of Sec. 4, "Hash Function", before interleaved coding),
 * partition-major (h_out[j * B + i] = pilot of bucket i of partition j), into h_out (host, cap
 * entries).  Needs PHOBIC_FLAG_KEEP_PILOTS at build time; PHOBIC_E_INVALID without it or when cap
 * is below K * B. */
phobic_status phobic_get_pilots(const phobic_mphf* h, uint32_t* h_out, uint64_t cap);

/* Per-phase times of the build that produced h (zeros for deserialized handles; for members of a
 * batch, the times of the whole batch, with hashing, partitioning and bucketing in bucket_sort_ms). */
phobic_status phobic_get_build_info(const phobic_mphf* h, phobic_build_info* out);

/* Serializes h into h_buf (host): the partition offsets as differences to their expectation
 * (Sec. 4, "Encoding the offsets") and the interleaved pilot encoders (Sec. 4.1), little-endian
 * 64-bit words.  *inout_bytes holds the capacity on entry and the image size on return; with
 * h_buf = NULL only the size is returned; a smaller capacity gives PHOBIC_E_INVALID. */
phobic_status phobic_serialize(const phobic_mphf* h, void* h_buf, uint64_t* inout_bytes);

/* Rebuilds a handle on the current device from an image made by phobic_serialize (the layout of
 * Sec. 4 and Sec. 4.1 written there).  Every field, section extent, unary stream and select entry is
 * checked on the host first; an inconsistent image gives PHOBIC_E_FORMAT and no handle. */
phobic_status phobic_deserialize(const void* h_buf, uint64_t bytes, void* hip_stream, phobic_mphf** out);

/* Hashing and partitioning alone, for parity checks: hashes and partitions the keys.  d_offsets gets K + 1
 * key offsets, d_codes gets 2 n words: partition j's codes (hi, lo) at [2 d_offsets[j], 2
 * d_offsets[j+1]) in unspecified order.  K = max(1, ceil(n / P)). */
phobic_status phobic_partition_u64(const uint64_t* d_keys, uint64_t n, const phobic_params* params,
                                   void* hip_stream, uint64_t* d_offsets, uint64_t* d_codes);

/* Launch shape of the pilot search: waves_per_group wavefronts per workgroup, each working on one
 * partition at a time; with groups_per_cu > 0 the search runs persistently (groups_per_cu
 * workgroups per compute unit pulling items_per_grab partitions at a time from an atomic queue),
 * with 0 it launches one wavefront per partition.  The shape never changes a result. */
typedef struct {
  uint32_t waves_per_group; /* 1, 2, 4 or 8 */
  uint32_t groups_per_cu;   /* 0 = one wavefront per partition; else persistent */
  uint32_t items_per_grab;  /* partitions taken per queue access (persistent mode), >= 1 */
  uint32_t reserved;
} phobic_search_config;

/* Sets the search shape used by later builds on the calling process (all devices).  The default is
 * one wavefront per workgroup, one wavefront per partition ({1, 0, 1, 0}). */
phobic_status phobic_set_search_config(const phobic_search_config* cfg);
phobic_status phobic_get_search_config(phobic_search_config* out);

/* Builds `count` independent MPHFs together: MPHF t is built from the h_counts[t] distinct keys at
 * the device pointer h_key_ptrs[t] (both arrays are host arrays of `count` entries), all with the
 * same params (alpha must be 1).  Each member follows the construction of Sec. 3, Sec. 4 and
 * Sec. 4.1 exactly as phobic_build_u64 does; the partition independence that makes this possible is
 * the one Sec. 4.2 relies on for its parallel search.  Every handle outs[t] is identical -- pilots, image, positions --
 * to what phobic_build_u64 returns for the same keys.  Hashing, partitioning and bucketing run over
 * the concatenated key sets; the pilot search is one persistent launch over all (MPHF, partition)
 * items; encoding runs for all MPHFs in a handful of launches.  The handles share one device
 * allocation that is released with the last of them.  On failure every outs[t] is NULL and
 * phobic_last_error() names the first failing MPHF. */
phobic_status phobic_build_batch_u64(const uint64_t* const* h_key_ptrs, const uint64_t* h_counts, uint32_t count,
                                     const phobic_params* params, void* hip_stream, phobic_mphf** outs);

/* ---- Serving: resident MPHFs, build and query requests under an HBM budget ----------------------
 * A server keeps the MPHFs it built resident on the device and runs requests on `workers` HIP
 * streams at once.  Requests are admitted in arrival order as workers and memory free up: a build
 * is admitted when its estimated device memory (32 bytes per key plus 64 MiB) fits in what the
 * budget leaves after resident images and builds in flight; a query needs no memory of its own.
 * Continuous batching: a worker that picks up queries takes up to max_query_batch pending ones (any
 * MPHFs) into one launch, and a worker that picks up builds takes up to max_build_batch admissible
 * ones into one batched build.  Neither changes any pilot, image or position.  The caller owns all
 * key and output buffers and keeps them valid until the request completes.  All calls are
 * thread-safe. */
typedef struct phobic_server phobic_server;

typedef struct {
  uint64_t hbm_budget_bytes; /* device memory for builds in flight and resident images */
  uint32_t workers;          /* requests in flight at once, one HIP stream each, >= 1 */
  uint32_t max_query_batch;  /* queries per launch, >= 1 (1 = no query batching) */
  uint32_t max_build_batch;  /* builds per batched build, >= 1 (1 = no build batching) */
  uint32_t query_workers;    /* workers that take queries only, < workers (0 = every worker takes both) */
} phobic_server_config;

enum { PHOBIC_REQ_BUILD = 0, PHOBIC_REQ_QUERY = 1 };

typedef struct {
  uint64_t request_id;
  uint64_t mphf_id;  /* builds: the id of the new MPHF (= request_id); queries: the queried MPHF */
  uint64_t n;        /* keys of the request */
  int32_t status;    /* phobic_status of the request */
  uint32_t kind;     /* PHOBIC_REQ_BUILD or PHOBIC_REQ_QUERY */
  uint32_t batch;    /* requests that ran in the same launch or batched build */
  uint32_t reserved;
  double submit_s, start_s, done_s; /* seconds on the server's steady clock */
} phobic_request_result;

typedef struct {
  uint64_t resident_mphfs;
  uint64_t resident_bytes;
  uint64_t reserved_bytes;   /* estimates of builds in flight */
  uint64_t peak_bytes;       /* peak of resident + reserved */
  uint64_t query_launches, build_launches;
  uint64_t completed, pending;
} phobic_server_stats;

phobic_status phobic_server_create(const phobic_server_config* cfg, const phobic_params* params,
                                   phobic_server** out);
/* Queues a build of the n keys at d_keys; *request_id is also the id of the MPHF it creates, so
 * queries against it may be queued before it completes (they wait for it). */
phobic_status phobic_server_submit_build(phobic_server* s, const uint64_t* d_keys, uint64_t n,
                                         uint64_t* request_id);
/* Queues a query of the n keys at d_keys against MPHF mphf_id; positions go to d_pos.  Fails at
 * once (PHOBIC_E_INVALID) for an unknown or released MPHF and for one whose build has already
 * failed; a query queued before its build fails completes with status PHOBIC_E_INVALID. */
phobic_status phobic_server_submit_query(phobic_server* s, uint64_t mphf_id, const uint64_t* d_keys, uint64_t n,
                                         uint64_t* d_pos, uint64_t* request_id);
/* Moves up to cap completed results into out (completion order); waits up to wait_ms for one. */
phobic_status phobic_server_poll(phobic_server* s, phobic_request_result* out, uint32_t cap, uint32_t* got,
                                 uint32_t wait_ms);
/* The resident MPHF mphf_id (borrowed; valid until released), or NULL. */
const phobic_mphf* phobic_server_mphf(phobic_server* s, uint64_t mphf_id);
/* Frees a resident MPHF once no queued or running query uses it. */
phobic_status phobic_server_release(phobic_server* s, uint64_t mphf_id);
phobic_status phobic_server_get_stats(phobic_server* s, phobic_server_stats* out);
double phobic_server_now(phobic_server* s); /* the server's clock, seconds */
/* Waits for every queued request, then frees the resident MPHFs and the server. */
void phobic_server_destroy(phobic_server* s);

/* Releases a handle.  The image goes back to the library's pool in the order of the default (NULL)
 * stream, which follows the work already queued on blocking streams; queries still queued on a
 * non-blocking stream must have completed, or been joined into the default stream, before the call. */
void phobic_free(phobic_mphf* h);
const char* phobic_status_str(phobic_status s);
const char* phobic_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PHOBIC_H */
