// CPU run of the pilot-search kernel logic (search_partition of the library's search.hip) on one
// partition, for the emulated-search test.  Built with g++ against the host stand-in of
// <hip/hip_runtime.h> in this folder, with AddressSanitizer: the wavefront's LDS is one heap block
// of exactly the size the library would give it, so any access outside it is reported.
//
// Usage: search_emu MODE IN OUT
//   MODE 0: tables up to 4096 slots; 1: larger tables (several scan passes); 2: wide partitions
//   (bucket list in global memory)
//   IN:  u64 m, limit, B, nj, nb; u64 fingerprints[nj] (processing order); u32 entries[nb]
//        (size << 16 | bucket, processing order)
//   OUT: u32 pilots[B]; u32 error bits
#include <vector>

#include SEARCH_SRC

// the kernels' dynamic LDS symbol (the CPU run hands search_partition its own block instead)
namespace phobic {
namespace {
alignas(16) uint32_t lds32[4];
}  // namespace
}  // namespace phobic

EmuIdx threadIdx, blockIdx, blockDim, gridDim;
EmuWave* emu_wave;
namespace phobic {
void set_error(const std::string&) {}
phobic_status fail(phobic_status s, const std::string&) { return s; }
}  // namespace phobic

using namespace phobic;

namespace {
SearchArgs g_sa;
uint32_t* g_lds;
int g_mode;
bool g_done[64];

void lane_main() {
  const unsigned me = threadIdx.x;
  if (g_mode == 0)
    search_partition<false, false>(g_sa, 0, g_lds, me);
  else if (g_mode == 1)
    search_partition<true, false>(g_sa, 0, g_lds, me);
  else
    search_partition<true, true>(g_sa, 0, g_lds, me);
  g_done[me] = true;
}
}  // namespace

int main(int argc, char** argv) {
  if (argc != 4) {
    std::fprintf(stderr, "usage: search_emu MODE IN OUT\n");
    return 2;
  }
  g_mode = std::atoi(argv[1]);
  FILE* f = std::fopen(argv[2], "rb");
  uint64_t h[5];
  if (!f || std::fread(h, 8, 5, f) != 5) return 3;
  const uint32_t m = (uint32_t)h[0], B = (uint32_t)h[2];
  const uint64_t limit = h[1], nj = h[3], nb = h[4];
  std::vector<uint64_t> fp(nj);
  std::vector<uint32_t> blist(B, 0);
  if (std::fread(fp.data(), 8, nj, f) != nj || std::fread(blist.data(), 4, nb, f) != nb) return 3;
  std::fclose(f);
  uint32_t maxb = 1;
  for (uint64_t i = 0; i < nb; i++) maxb = std::max<uint32_t>(maxb, blist[i] >> 16);
  std::vector<uint64_t> off = {0, nj}, toff = {0, m};
  std::vector<uint32_t> nbk = {(uint32_t)nb};
  std::vector<uint32_t> pilots(B, 0xDEADBEEFu);
  std::vector<uint32_t> err(1, 0);
  const bool wide = g_mode == 2;
  SearchArgs& sa = g_sa;
  sa = SearchArgs{};
  sa.fp = fp.data();
  sa.off = off.data();
  sa.toff = toff.data();
  sa.blist = blist.data();
  sa.nbk = nbk.data();
  sa.pilots = pilots.data();
  sa.err = err.data();
  sa.K = 1;
  sa.limit = limit;
  sa.B = B;
  // the LDS layout the library builds for these sizes
  size_search_lds(sa, std::max<uint32_t>(m, 1), maxb, B, wide);
  g_lds = (uint32_t*)std::aligned_alloc(16, sa.wave_lds);
  std::memset(g_lds, 0xA5, sa.wave_lds);  // LDS starts with garbage

  static EmuWave wave;
  emu_wave = &wave;
  constexpr size_t kStack = 1 << 16;
  std::vector<char> stacks(64 * kStack);
  for (unsigned l = 0; l < 64; l++) {
    getcontext(&wave.lane[l]);
    wave.lane[l].uc_stack.ss_sp = stacks.data() + (size_t)l * kStack;
    wave.lane[l].uc_stack.ss_size = kStack;
    wave.lane[l].uc_link = &wave.sched;
    makecontext(&wave.lane[l], lane_main, 0);
  }
  // each round resumes every lane up to its next collective (or its end); all lanes must end in the
  // same round, as a wavefront's lanes leave a uniform function together
  for (;;) {
    unsigned ended = 0;
    for (unsigned l = 0; l < 64; l++) {
      if (g_done[l]) {
        ended++;
        continue;
      }
      threadIdx.x = l;
      swapcontext(&wave.sched, &wave.lane[l]);
    }
    unsigned now = 0;
    for (unsigned l = 0; l < 64; l++) now += g_done[l];
    if (now == 64) break;
    if (now != 0 || ended != 0) {
      std::fprintf(stderr, "lanes left the kernel at different collectives\n");
      return 4;
    }
  }
  std::free(g_lds);
  FILE* o = std::fopen(argv[3], "wb");
  std::fwrite(pilots.data(), 4, B, o);
  std::fwrite(err.data(), 4, 1, o);
  std::fclose(o);
  return 0;
}
