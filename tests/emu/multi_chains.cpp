// Test-only: batches of two lattices swept together on the host emulation (emu_hip.h), through
// dqmc_sweep_multi and through a recorded graph (dqmc_graph_create / dqmc_graph_launch, three
// replays), each compared bit for bit (fields and observables) with the same batches swept one
// at a time with dqmc_sweep.  Square L1 x L1 and L2 x L2, U = 4, dtau = 0.1, BETA; exit status 3
// if any differs.
// usage: multi_chains L1 L2 BETA CHAINS SWEEPS1 SWEEPS2
#include "emu_hip.h"
#include "dqmc.h"
#include "dqmc_device.hpp"

void emu_call_kernel(const void* fn, void** params) {
  auto k = reinterpret_cast<void (*)(dqmc::KArgs)>(const_cast<void*>(fn));
  k(*reinterpret_cast<dqmc::KArgs*>(params[0]));
}

static std::vector<double> square_hopping(int L) {
  const int n = L * L;
  std::vector<double> T((size_t)n * n, 0.0);
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x) {
      const int i = x + L * y;
      const int nb[2] = {((x + 1) % L) + L * y, x + L * ((y + 1) % L)};
      for (int j : nb) {
        T[(size_t)i * n + j] += -1.0;
        T[(size_t)j * n + i] += -1.0;
      }
    }
  return T;
}

struct Set {
  std::vector<double> T;
  dqmc_model m{};
  char* w = nullptr;
  dqmc_batch* b = nullptr;
  int n = 0, ns = 0, chains = 0;
};

static void make(Set& s, int L, double beta, int chains) {
  s.T = square_hopping(L);
  s.n = L * L;
  s.ns = (int)std::lround(beta / 0.1);
  s.chains = chains;
  s.m.n_sites = s.n; s.m.hopping = s.T.data(); s.m.U = 4.0; s.m.dtau = 0.1; s.m.n_slices = s.ns;
  s.m.stab_every = 10; s.m.precision = DQMC_FP64;
  std::vector<uint64_t> seeds(chains);
  for (int c = 0; c < chains; ++c) seeds[c] = 0xB0000ull + 31 * c + L;
  const size_t ws = dqmc_workspace_bytes(&s.m, chains);
  s.w = (char*)std::aligned_alloc(256, (ws + 255) & ~(size_t)255);
  std::memset(s.w, 0xA5, ws);
  if (dqmc_init_chains(&s.b, &s.m, chains, nullptr, seeds.data(), s.w, ws, nullptr)) std::exit(1);
}

static std::vector<char> state(Set& s) {
  std::vector<dqmc_obs> o(s.chains);
  dqmc_measure(s.b, o.data(), nullptr, nullptr);
  std::vector<int8_t> f((size_t)s.chains * s.ns * s.n);
  dqmc_get_fields(s.b, f.data(), nullptr);
  std::vector<char> out((const char*)o.data(), (const char*)(o.data() + o.size()));
  out.insert(out.end(), (const char*)f.data(), (const char*)(f.data() + f.size()));
  return out;
}

int main(int argc, char** argv) {
  if (argc != 7) return 2;
  const int L1 = std::atoi(argv[1]), L2 = std::atoi(argv[2]);
  const double beta = std::atof(argv[3]);
  const int chains = std::atoi(argv[4]), s1 = std::atoi(argv[5]), s2 = std::atoi(argv[6]);
  int bad = 0;
  // sweep_multi against one batch at a time
  {
    Set a, b, ea, eb;
    make(a, L1, beta, chains); make(b, L2, beta, chains);
    make(ea, L1, beta, chains); make(eb, L2, beta, chains);
    dqmc_batch* bs[2] = {a.b, b.b};
    const int32_t ns[2] = {s1, s2};
    if (dqmc_sweep_multi(bs, ns, 2, nullptr)) return 1;
    dqmc_sweep(ea.b, s1, nullptr);
    dqmc_sweep(eb.b, s2, nullptr);
    const bool same = state(a) == state(ea) && state(b) == state(eb);
    std::printf("sweep_multi: %s\n", same ? "same" : "DIFFERENT");
    bad += !same;
  }
  // a recorded graph, three replays
  {
    Set a, b, ea, eb;
    make(a, L1, beta, chains); make(b, L2, beta, chains);
    make(ea, L1, beta, chains); make(eb, L2, beta, chains);
    dqmc_batch* bs[2] = {a.b, b.b};
    const int32_t ns[2] = {s1, s2};
    dqmc_graph* g = nullptr;
    if (dqmc_graph_create(&g, bs, ns, 2)) return 1;
    for (int rep = 0; rep < 3; ++rep) {
      if (dqmc_graph_launch(g, nullptr)) return 1;
      dqmc_sweep(ea.b, s1, nullptr);
      dqmc_sweep(eb.b, s2, nullptr);
      const bool same = state(a) == state(ea) && state(b) == state(eb);
      std::printf("graph replay %d: %s\n", rep, same ? "same" : "DIFFERENT");
      bad += !same;
    }
    dqmc_graph_destroy(g);
  }
  return bad ? 3 : 0;
}
