// Test-only: the Ising C ABI (include/ising.h) on the host emulation (emu_hip.h).  Reads seeds.bin
// (uint64 [n_chains]) from DIR, runs ising_init (spins drawn from the seeds) and one ising_sweep
// launch of N_SWEEPS measured sweeps with the per-sweep series, and writes spins.bin
// (int8 [n_chains][L*L]), series.bin (int32 [n_chains][N_SWEEPS][2]) and stats.bin (ising_obs).
// usage: ising_chains DIR L T N_CHAINS N_SWEEPS
#include "emu_hip.h"
#include "ising.h"

void emu_call_kernel(const void*, void**) {
  std::fprintf(stderr, "ising_chains: unexpected launch through a kernel pointer\n");
  std::abort();
}

int main(int argc, char** argv) {
  if (argc != 6) return 2;
  const std::string dir = argv[1];
  const int L = std::atoi(argv[2]);
  const double T = std::atof(argv[3]);
  const int n = std::atoi(argv[4]), sweeps = std::atoi(argv[5]);
  std::vector<uint64_t> seeds(n);
  FILE* f = std::fopen((dir + "/seeds.bin").c_str(), "rb");
  if (!f || std::fread(seeds.data(), 8, n, f) != (size_t)n) return 2;
  std::fclose(f);
  const size_t ws = ising_workspace_bytes(L, n);
  char* w = (char*)std::aligned_alloc(256, (ws + 255) & ~(size_t)255);
  std::memset(w, 0xA5, ws);
  ising_batch* b = nullptr;
  int st = ising_init(&b, L, 1.0, T, n, nullptr, seeds.data(), w, ws, nullptr);
  if (st) { std::fprintf(stderr, "ising_init %d\n", st); return 1; }
  std::vector<int32_t> series((size_t)n * sweeps * 2);
  st = ising_sweep(b, sweeps, 1, series.data(), nullptr);
  if (st) { std::fprintf(stderr, "ising_sweep %d\n", st); return 1; }
  std::vector<ising_obs> obs(n);
  std::vector<int8_t> spins((size_t)n * L * L);
  ising_stats(b, obs.data(), nullptr);
  ising_get_spins(b, spins.data(), nullptr);
  auto put = [&](const char* name, const void* p, size_t bytes) {
    FILE* o = std::fopen((dir + "/" + name).c_str(), "wb");
    std::fwrite(p, 1, bytes, o);
    std::fclose(o);
  };
  put("spins.bin", spins.data(), spins.size());
  put("series.bin", series.data(), series.size() * 4);
  put("stats.bin", obs.data(), obs.size() * sizeof(ising_obs));
  ising_destroy(b);
  std::free(w);
  return 0;
}
