// Host side of the C ABI: parameters, planning (bucket-function table, Rice parameter), handles,
// serialization and error reporting.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <algorithm>
#include <vector>

#include "phobic_internal.h"

namespace phobic {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

phobic_status fail(phobic_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

uint64_t num_partitions(uint64_t n, uint32_t P) {
  uint64_t K = (n + P - 1) / P;  // expected partition size P (Sec. 4)
  return K ? K : 1;
}

phobic_status validate_params(const phobic_params* p, uint32_t* B) {
  if (!p) return fail(PHOBIC_E_INVALID, "params is null");
  if (p->partition_size < 1) return fail(PHOBIC_E_INVALID, "partition_size must be >= 1");
  if (!(p->lambda > 0.0) || !std::isfinite(p->lambda)) return fail(PHOBIC_E_INVALID, "lambda must be > 0");
  if (p->alpha_den == 0 || p->alpha_num == 0 || p->alpha_num > p->alpha_den)
    return fail(PHOBIC_E_INVALID, "alpha must be in (0, 1]");
  if (p->coding > 1) return fail(PHOBIC_E_INVALID, "unknown coding");
  if (p->bucket_function > PHOBIC_BF_UNIFORM) return fail(PHOBIC_E_INVALID, "unknown bucket function");
  if (p->reserved != 0) return fail(PHOBIC_E_INVALID, "params.reserved must be 0");
  if (p->pilot_limit > 0xFFFFFFFFULL) return fail(PHOBIC_E_INVALID, "pilot_limit exceeds 2^32 - 1");
  double b = std::ceil((double)p->partition_size / p->lambda);  // B = P / lambda (Sec. 4.1)
  if (b < 1.0 || b > 65535.0) return fail(PHOBIC_E_INVALID, "B = ceil(P / lambda) must be in [1, 65535]");
  *B = (uint32_t)b;
  // mixed interleaved coding (Sec. 4.1: Compact for the first, largest buckets, Golomb-Rice for the
  // rest) is a variant of the Rice image; an all-Compact image has no Rice encoders to replace
  if (p->coding == PHOBIC_IC_RICE && p->n_compact > *B)
    return fail(PHOBIC_E_INVALID, "n_compact must be at most B");
  if (p->coding == PHOBIC_IC_COMPACT && p->n_compact != 0 && p->n_compact != *B)
    return fail(PHOBIC_E_INVALID, "n_compact must be 0 or B with Compact coding");
  return PHOBIC_OK;
}

// beta_* (Sec. 3.2), beta_eps with eps = lambda / (5 sqrt(P)) (Thm. 2, App. C.1), and the functions
// of related work it is compared with (Sec. 3.1): PTHash's skewed one (the first 60% of the hash
// range spread over the first 30% of the buckets, the rest over the others) and CHD's uniform one.
// Rescaled to gamma_alpha for alpha < 1 (App. B); tabulated at 2049 points as round(2^32 gamma(k / 2048)).
static double beta_star(double x) { return x >= 1.0 ? 1.0 : x + (1.0 - x) * std::log1p(-x); }

void bucket_table(double lambda, uint32_t P, uint32_t an, uint32_t ad, uint32_t fn, uint64_t* T) {
  double eps = lambda / (5.0 * std::sqrt((double)P));
  if (eps > 1.0) eps = 1.0;
  auto gamma = [eps, fn](double x) {
    switch (fn) {
      case PHOBIC_BF_BETA_STAR: return beta_star(x);
      case PHOBIC_BF_SKEW: return x <= 0.6 ? 0.5 * x : 0.3 + 1.75 * (x - 0.6);
      case PHOBIC_BF_UNIFORM: return x;
      default: return eps * x + (1.0 - eps) * beta_star(x);
    }
  };
  const double alpha = (double)an / (double)ad;
  const double norm = gamma(alpha);
  for (uint32_t k = 0; k <= kTableIntervals; k++) {
    const double x = (double)k / kTableIntervals;
    const double g = an == ad ? gamma(x) : gamma(alpha * x) / norm;
    T[k] = (uint64_t)std::llround(std::ldexp(g, 32));
  }
  T[0] = 0;
  T[kTableIntervals] = 1ULL << 32;
}

// Golomb-Rice parameter by Kiely's rule for a geometric source of mean mu (Sec. 4.1):
// b = max(0, 1 + floor(log2(ln(phi - 1) / ln(mu / (mu + 1))))).
static uint32_t rice_of_mean(double mu) {
  const double phi = (1.0 + std::sqrt(5.0)) / 2.0;
  double b = 1.0 + std::floor(std::log2(std::log(phi - 1.0) / std::log(mu / (mu + 1.0))));
  if (b < 0.0) b = 0.0;
  if (b > 32.0) b = 32.0;
  return (uint32_t)b;
}

uint32_t rice_parameter(uint64_t sum, uint64_t count) {
  if (sum == 0 || count == 0) return 0;
  return rice_of_mean((double)sum / (double)count);
}

// mu_t = the smallest positive double with rice_of_mean(mu) >= t + 1, by bisection over the bit
// patterns of positive doubles (ordered like their values, and the formula does not decrease with mu).
const RiceThresholds& rice_thresholds() {
  static RiceThresholds th;
  static std::once_flag once;
  std::call_once(once, [] {
    auto as_double = [](uint64_t bits) {
      double d;
      std::memcpy(&d, &bits, 8);
      return d;
    };
    for (uint32_t t = 0; t < 32; t++) {
      uint64_t lo = 1, hi = 0x4340000000000000ULL;  // 2^53, where the parameter is 32
      while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (rice_of_mean(as_double(mid)) >= t + 1) hi = mid; else lo = mid + 1;
      }
      th.mu[t] = as_double(lo);
    }
  });
  return th;
}

// Device copies of bucket-function tables, one per (device, lambda, P, alpha); they live until the
// process ends, so handles only borrow them.
namespace {
struct TableKey {
  int device;
  uint64_t lambda_bits;
  uint32_t P, an, ad, fn;
  bool operator<(const TableKey& o) const {
    return std::tie(device, lambda_bits, P, an, ad, fn) < std::tie(o.device, o.lambda_bits, o.P, o.an, o.ad, o.fn);
  }
};
std::mutex g_table_mu;
std::map<TableKey, uint64_t*> g_tables;
}  // namespace

hipError_t pool_alloc(void** p, size_t bytes, hipStream_t st) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  static std::mutex mu;
  static std::vector<hipMemPool_t> pools;
  hipMemPool_t pool = nullptr;
  {
    std::lock_guard<std::mutex> lock(mu);
    if ((size_t)dev >= pools.size()) pools.resize((size_t)dev + 1, nullptr);
    if (!pools[dev]) {
      hipMemPoolProps props{};
      props.allocType = hipMemAllocationTypePinned;
      props.handleTypes = hipMemHandleTypeNone;
      props.location.type = hipMemLocationTypeDevice;
      props.location.id = dev;
      hipMemPool_t created = nullptr;
      e = hipMemPoolCreate(&created, &props);
      if (e != hipSuccess) return e;
      uint64_t keep = kPoolKeepBytes;
      e = hipMemPoolSetAttribute(created, hipMemPoolAttrReleaseThreshold, &keep);
      if (e != hipSuccess) {
        (void)hipMemPoolDestroy(created);
        return e;
      }
      pools[dev] = created;
    }
    pool = pools[dev];
  }
  return hipMallocFromPoolAsync(p, bytes, pool, st);
}

size_t max_lds_per_group() {
  static std::mutex mu;
  static std::map<int, size_t> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 64 * 1024;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) v = 64 * 1024;
  cache[dev] = (size_t)v;
  return (size_t)v;
}

phobic_status upload_table(phobic_mphf* h, hipStream_t st) {
  TableKey key{h->device, 0, h->prm.partition_size, h->prm.alpha_num, h->prm.alpha_den, h->prm.bucket_function};
  std::memcpy(&key.lambda_bits, &h->prm.lambda, 8);
  std::lock_guard<std::mutex> lock(g_table_mu);
  auto it = g_tables.find(key);
  if (it != g_tables.end()) {
    h->d_table = it->second;
    return PHOBIC_OK;
  }
  std::vector<uint64_t> T(kTableIntervals + 1);
  bucket_table(h->prm.lambda, h->prm.partition_size, h->prm.alpha_num, h->prm.alpha_den, h->prm.bucket_function,
               T.data());
  uint64_t* d = nullptr;
  PHOBIC_HIP(hipMalloc(&d, T.size() * sizeof(uint64_t)));
  hipError_t e = hipMemcpyAsync(d, T.data(), T.size() * sizeof(uint64_t), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);  // T is a local vector
  if (e != hipSuccess) {
    (void)hipFree(d);
    return fail(PHOBIC_E_DEVICE, std::string("bucket table upload: ") + hipGetErrorString(e));
  }
  g_tables[key] = d;
  h->d_table = d;
  return PHOBIC_OK;
}

// Header words of an image; the section layout follows from the sizes (see the format notes).
std::vector<uint64_t> make_header(uint64_t n, uint64_t K, uint32_t B, const phobic_params& prm, uint64_t total,
                                  int64_t dmin, uint32_t woff, uint64_t data_bits, uint64_t unary_bits, uint64_t R) {
  std::vector<uint64_t> hdr(kHeaderWords, 0);
  uint64_t lambda_bits;
  std::memcpy(&lambda_bits, &prm.lambda, 8);
  fill_header(hdr.data(), n, K, B, prm.partition_size, lambda_bits,
              (uint64_t)prm.alpha_num | ((uint64_t)prm.alpha_den << 32),
              prm.coding | ((uint64_t)prm.bucket_function << 8), prm.hash_seed, total, dmin, woff, data_bits,
              unary_bits, R, prm.coding == PHOBIC_IC_RICE ? prm.n_compact : 0);
  return hdr;
}

void fill_query_args(phobic_mphf* h) {
  const std::vector<uint64_t>& H = h->header;
  QueryArgs& a = h->qa;
  a.img = h->d_image;
  a.table = h->d_table;
  a.n = H[kHN];
  a.K = H[kHK];
  a.R = H[kHR];
  a.total = H[kHTotal];
  a.dmin = (int64_t)H[kHDmin];
  a.sec_off = H[kHSecOff];
  a.sec_enc = H[kHSecEnc];
  a.sec_data = H[kHSecData];
  a.sec_unary = H[kHSecUnary];
  a.sec_sel = H[kHSecSel];
  a.sec_remap = H[kHSecRemap];
  a.seed = H[kHSeed];
  a.B = (uint32_t)H[kHB];
  a.woff = (uint32_t)H[kHWoff];
  a.coding = (uint32_t)(H[kHCoding] & 0xFF);
  a.wremap = (uint32_t)H[kHWremap];
  a.ncompact = (uint32_t)H[kHNcompact];
}

static uint64_t host_bits(const uint64_t* w, uint64_t pos, uint32_t width) {
  if (width == 0) return 0;
  uint64_t idx = pos >> 6;
  uint32_t sh = (uint32_t)(pos & 63);
  uint64_t v = w[idx] >> sh;
  if (sh + width > 64) v |= w[idx + 1] << (64 - sh);
  return width == 64 ? v : (v & ((1ULL << width) - 1));
}

static uint32_t host_bit_length(uint64_t v) { return v ? 64 - __builtin_clzll(v) : 0; }

// Checks that an image is internally consistent, so the query kernel never reads outside it.
static phobic_status check_image(const uint64_t* w, uint64_t nwords) {
  auto bad = [](const char* what) { return fail(PHOBIC_E_FORMAT, std::string("malformed image: ") + what); };
  if (nwords < kHeaderWords || w[kHMagic] != kMagic) return bad("magic");
  if (w[kHWords] != nwords) return bad("length");
  const uint64_t n = w[kHN], K = w[kHK], B = w[kHB], total = w[kHTotal];
  const uint64_t coding = w[kHCoding] & 0xFF, bfn = w[kHCoding] >> 8;
  if (K == 0 || B == 0 || B > 65535 || coding > 1 || bfn > PHOBIC_BF_UNIFORM || total < n) return bad("sizes");
  const uint64_t c = w[kHNcompact];  // Compact encoders before the Rice ones (Rice images only)
  if (c > B || (coding != PHOBIC_IC_RICE && c != 0)) return bad("mixed coding");
  const uint32_t an = (uint32_t)w[kHAlpha], ad = (uint32_t)(w[kHAlpha] >> 32);
  if (an == 0 || ad == 0 || an > ad || w[kHP] == 0 || w[kHP] > 0xFFFFFFFFULL) return bad("parameters");
  double lambda;
  std::memcpy(&lambda, &w[kHLambda], 8);
  if (!(lambda > 0.0) || !std::isfinite(lambda) || (uint64_t)std::ceil((double)w[kHP] / lambda) != B)
    return bad("lambda");
  if (K != num_partitions(n, (uint32_t)w[kHP])) return bad("partition count");
  if (w[kHWoff] > 64 || w[kHWremap] > 64) return bad("widths");
  const uint64_t so = w[kHSecOff], se = w[kHSecEnc], sd = w[kHSecData], su = w[kHSecUnary], ss = w[kHSecSel],
                 sr = w[kHSecRemap];
  if (so != kHeaderWords) return bad("section order");
  if (se != so + ((K + 1) * w[kHWoff] + 63) / 64 + 1 || sd != se + B + 1 || su < sd || ss < su || sr < ss ||
      sr > nwords)
    return bad("section layout");
  // offsets: 0 first, total last, non-decreasing
  uint64_t prev = 0;
  for (uint64_t j = 0; j <= K; j++) {
    uint64_t o = phobic::expected_offset_host(j, w[kHR]) + w[kHDmin] + host_bits(w + so, j * w[kHWoff], (uint32_t)w[kHWoff]);
    if ((j == 0 && o != 0) || o < prev || (j == K && o != total)) return bad("offsets");
    prev = o;
  }
  // encoders: payload inside the data section
  const uint64_t data_bits = (su - sd - 1) * 64;
  for (uint64_t i = 0; i < B; i++) {
    const uint64_t e = w[se + i];
    const uint32_t wd = (uint32_t)(e & 0xFF);
    if (wd > 32 || (e >> 8) + (uint64_t)wd * K > data_bits) return bad("encoder table");
  }
  const uint64_t nvals = K * (B - c);  // values of the Rice encoders: one one each in the unary stream
  if (coding == PHOBIC_IC_RICE) {
    const uint64_t ubits = w[kHUbits];
    if (su + (ubits + 63) / 64 + 1 != ss) return bad("unary length");
    uint64_t ones = 0;
    for (uint64_t i = 0; i < (ubits + 63) / 64; i++) ones += __builtin_popcountll(w[su + i]);
    if (ones != nvals || w[ss - 1] != 0) return bad("unary stream");
    const uint64_t nsel = (nvals + kSelBlock - 1) / kSelBlock;
    if (ss + nsel + 1 != sr) return bad("select length");
    // every entry must hold exactly the position of one number kSelBlock s and the distances to ones
    // kSelBlock s + kSelSub k: positions of every kSelSub-th one first
    std::vector<uint64_t> p64((nvals + kSelSub - 1) / kSelSub);
    uint64_t seen = 0, s_next = 0;
    for (uint64_t i = 0; i < (ubits + 63) / 64 && s_next < p64.size(); i++) {
      uint64_t x = w[su + i];
      while (x && s_next < p64.size()) {
        const uint64_t c = (uint64_t)__builtin_popcountll(x);
        const uint64_t want = s_next * kSelSub;
        if (seen + c <= want) {
          seen += c;
          break;
        }
        for (uint64_t skip = want - seen; skip; skip--) x &= x - 1;  // drop ones before the target
        p64[s_next++] = i * 64 + (uint64_t)__builtin_ctzll(x);
        seen = want + 1;
        x &= x - 1;
      }
    }
    if (s_next != p64.size()) return bad("select samples");
    constexpr uint32_t per = kSelBlock / kSelSub;
    for (uint64_t sb = 0; sb < nsel; sb++) {
      const uint64_t a0 = p64[sb * per];
      if (a0 >> 32) return bad("select range");
      uint64_t want = a0;
      for (uint32_t k = 1; k < per; k++) {
        const uint64_t idx = sb * per + k;
        const uint64_t rel = idx < p64.size() ? std::min<uint64_t>(p64[idx] - a0, kSelRelNone) : 0;
        want |= rel << (32 + 10 * (k - 1));
      }
      if (w[ss + sb] != want) return bad("select samples");
    }
  } else if (su != ss || ss != sr) {
    return bad("compact layout");
  }
  const uint64_t nremap = total - n;
  if (w[kHNremap] != nremap || (nremap && w[kHWremap] != (n > 1 ? host_bit_length(n - 1) : 0)))
    return bad("remap");
  const uint64_t want_end = sr + (nremap ? (nremap * w[kHWremap] + 63) / 64 + 1 : 0);
  if (want_end != nwords) return bad("remap length");
  for (uint64_t g = 0; g < nremap; g++)
    if (host_bits(w + sr, g * w[kHWremap], (uint32_t)w[kHWremap]) >= n) return bad("remap entries");
  return PHOBIC_OK;
}

}  // namespace phobic

using namespace phobic;

extern "C" void phobic_params_default(phobic_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->partition_size = 2500;
  p->coding = PHOBIC_IC_RICE;
  p->lambda = 7.0;
  p->alpha_num = 1;
  p->alpha_den = 1;
  p->hash_seed = 0x5EED;
}

extern "C" uint64_t phobic_size_bits(const phobic_mphf* h) { return h ? h->nwords * 64 : 0; }
extern "C" uint64_t phobic_num_keys(const phobic_mphf* h) { return h ? h->n : 0; }
extern "C" uint64_t phobic_num_partitions(const phobic_mphf* h) { return h ? h->K : 0; }
extern "C" uint32_t phobic_num_buckets(const phobic_mphf* h) { return h ? h->B : 0; }

extern "C" phobic_status phobic_get_pilots(const phobic_mphf* h, uint32_t* h_out, uint64_t cap) {
  if (!h || !h_out) return fail(PHOBIC_E_INVALID, "null argument");
  if (!h->d_pilots) return fail(PHOBIC_E_INVALID, "the handle was built without PHOBIC_FLAG_KEEP_PILOTS");
  const uint64_t K = h->K, B = h->B;
  if (cap < K * B) return fail(PHOBIC_E_INVALID, "output buffer too small");
  // the kept array is partition-major already
  PHOBIC_HIP(hipMemcpy(h_out, h->d_pilots, K * B * sizeof(uint32_t), hipMemcpyDeviceToHost));
  return PHOBIC_OK;
}

extern "C" phobic_status phobic_get_build_info(const phobic_mphf* h, phobic_build_info* out) {
  if (!h || !out) return fail(PHOBIC_E_INVALID, "null argument");
  *out = h->info;
  return PHOBIC_OK;
}

extern "C" phobic_status phobic_serialize(const phobic_mphf* h, void* h_buf, uint64_t* inout_bytes) {
  if (!h || !inout_bytes) return fail(PHOBIC_E_INVALID, "null argument");
  const uint64_t bytes = h->nwords * sizeof(uint64_t);
  if (!h_buf) {
    *inout_bytes = bytes;
    return PHOBIC_OK;
  }
  if (*inout_bytes < bytes) {
    *inout_bytes = bytes;
    return fail(PHOBIC_E_INVALID, "buffer too small");
  }
  PHOBIC_HIP(hipMemcpy(h_buf, h->d_image, bytes, hipMemcpyDeviceToHost));
  *inout_bytes = bytes;
  return PHOBIC_OK;
}

extern "C" phobic_status phobic_deserialize(const void* h_buf, uint64_t bytes, void* hip_stream, phobic_mphf** out) {
  if (!out) return fail(PHOBIC_E_INVALID, "out is null");
  *out = nullptr;
  if (!h_buf || bytes % 8 != 0) return fail(PHOBIC_E_FORMAT, "image size is not a whole number of words");
  const uint64_t nwords = bytes / 8;
  std::vector<uint64_t> w(nwords);
  std::memcpy(w.data(), h_buf, bytes);
  phobic_status s = check_image(w.data(), nwords);
  if (s != PHOBIC_OK) return s;
  hipStream_t st = (hipStream_t)hip_stream;
  auto h = new phobic_mphf();
  PHOBIC_HIP(hipGetDevice(&h->device));
  h->n = w[kHN];
  h->K = w[kHK];
  h->B = (uint32_t)w[kHB];
  h->header.assign(w.begin(), w.begin() + kHeaderWords);
  phobic_params_default(&h->prm);
  h->prm.partition_size = (uint32_t)w[kHP];
  std::memcpy(&h->prm.lambda, &w[kHLambda], 8);
  h->prm.alpha_num = (uint32_t)w[kHAlpha];
  h->prm.alpha_den = (uint32_t)(w[kHAlpha] >> 32);
  h->prm.coding = (uint32_t)(w[kHCoding] & 0xFF);
  h->prm.bucket_function = (uint32_t)(w[kHCoding] >> 8);
  h->prm.n_compact = (uint32_t)w[kHNcompact];
  h->prm.hash_seed = w[kHSeed];
  h->nwords = nwords;
  phobic_status r = upload_table(h, st);
  if (r != PHOBIC_OK) {
    phobic_free(h);
    return r;
  }
  hipError_t e = pool_alloc((void**)&h->d_image, bytes, st);
  if (e == hipSuccess) e = hipMemcpyAsync(h->d_image, w.data(), bytes, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    phobic_free(h);
    return fail(e == hipErrorOutOfMemory ? PHOBIC_E_OOM : PHOBIC_E_DEVICE, hipGetErrorString(e));
  }
  fill_query_args(h);
  *out = h;
  return PHOBIC_OK;
}

extern "C" void phobic_free(phobic_mphf* h) {
  if (!h) return;
  // the image comes from the library's stream-ordered pool; the null stream orders the release after
  // all work already enqueued on blocking streams.  Batch members share one allocation.
  if (h->shared)
    h->shared.reset();
  else if (h->d_image)
    (void)hipFreeAsync(h->d_image, nullptr);
  if (h->d_pilots) (void)hipFree(h->d_pilots);
  delete h;
}

extern "C" const char* phobic_status_str(phobic_status s) {
  switch (s) {
    case PHOBIC_OK: return "ok";
    case PHOBIC_E_INVALID: return "invalid argument";
    case PHOBIC_E_DUPLICATE: return "duplicate keys";
    case PHOBIC_E_OOM: return "out of memory";
    case PHOBIC_E_PILOT_OVERFLOW: return "pilot overflow";
    case PHOBIC_E_DEVICE: return "device error";
    case PHOBIC_E_FORMAT: return "malformed image";
    case PHOBIC_E_CAPACITY: return "capacity exceeded";
  }
  return "unknown status";
}

extern "C" const char* phobic_last_error(void) { return g_last_error.c_str(); }
