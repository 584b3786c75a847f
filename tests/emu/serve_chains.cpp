// Test-only: continuous batching on the host emulation (emu_hip.h).  Requests (square L x L,
// U = 4, dtau = 0.1) are served through slot re-initialisation (dqmc_init_slots) and per-chain
// sweep counts (dqmc_sweep_counts) in a batch of CAPACITY chains, TICK sweeps per launch; each
// result is then compared bit for bit with the same request run alone.  Exit status 3 if any
// differs.
// usage: serve_chains L BETA PREC(0|1) REFRESH N_REQ CAPACITY TICK [MAX_SWEEPS]
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

struct Result {
  dqmc_obs obs;
  std::vector<int8_t> fields;
};

int main(int argc, char** argv) {
  const int L = std::atoi(argv[1]);
  const double beta = std::atof(argv[2]);
  const int prec = std::atoi(argv[3]), refresh = std::atoi(argv[4]);
  const int n_req = std::atoi(argv[5]), cap = std::atoi(argv[6]), tick = std::atoi(argv[7]);
  const int n = L * L, ns = (int)std::lround(beta / 0.1);
  auto T = square_hopping(L);
  dqmc_model m{};
  m.n_sites = n; m.hopping = T.data(); m.U = 4.0; m.dtau = 0.1; m.n_slices = ns; m.stab_every = 10;
  m.refresh_every = refresh; m.precision = prec ? DQMC_FP32_WRAP : DQMC_FP64; m.drift_limit = 1.0;
  std::vector<uint64_t> seeds(n_req);
  std::vector<int> sweeps(n_req);
  for (int r = 0; r < n_req; ++r) {
    seeds[r] = 0x5EED0000ull + 977 * r;
    sweeps[r] = 2 + (r * 5) % 8;
    if (argc > 8) sweeps[r] = std::min(sweeps[r], std::atoi(argv[8]));
  }
  auto run_batch = [&](int nc, const uint64_t* sd, char** wout, dqmc_batch** bout) {
    const size_t ws = dqmc_workspace_bytes(&m, nc);
    char* w = (char*)std::aligned_alloc(256, (ws + 255) & ~(size_t)255);
    std::memset(w, 0xA5, ws);
    int st = dqmc_init_chains(bout, &m, nc, nullptr, sd, w, ws, nullptr);
    if (st) { std::fprintf(stderr, "init %d %s\n", st, dqmc_last_error()); std::exit(1); }
    *wout = w;
  };
  auto take = [&](dqmc_batch* b, int nc, int c) {
    std::vector<dqmc_obs> o(nc);
    dqmc_measure(b, o.data(), nullptr, nullptr);
    std::vector<int8_t> f((size_t)nc * ns * n);
    dqmc_get_fields(b, f.data(), nullptr);
    Result r;
    r.obs = o[c];
    r.fields.assign(f.begin() + (size_t)c * ns * n, f.begin() + (size_t)(c + 1) * ns * n);
    return r;
  };
  // served
  std::vector<Result> served(n_req);
  char* w = nullptr;
  dqmc_batch* b = nullptr;
  std::vector<uint64_t> init_seeds(cap);
  std::vector<int> slot_req(cap, -1), left(cap, 0);
  int next = 0;
  for (int c = 0; c < cap; ++c) {
    init_seeds[c] = next < n_req ? seeds[next] : 1;
    if (next < n_req) { slot_req[c] = next; left[c] = sweeps[next]; ++next; }
  }
  run_batch(cap, init_seeds.data(), &w, &b);
  int done = 0, ticks = 0;
  while (done < n_req) {
    std::vector<int32_t> counts(cap, 0);
    for (int c = 0; c < cap; ++c) counts[c] = slot_req[c] >= 0 ? std::min(tick, left[c]) : 0;
    int st = dqmc_sweep_counts(b, counts.data(), nullptr);
    if (st) { std::fprintf(stderr, "sweep_counts %d %s\n", st, dqmc_last_error()); return 1; }
    ++ticks;
    for (int c = 0; c < cap; ++c) {
      if (slot_req[c] < 0) continue;
      left[c] -= counts[c];
      if (left[c] > 0) continue;
      served[slot_req[c]] = take(b, cap, c);
      ++done;
      slot_req[c] = -1;
      if (next < n_req) {
        const int32_t s = c;
        st = dqmc_init_slots(b, &s, 1, nullptr, &seeds[next], nullptr);
        if (st) { std::fprintf(stderr, "init_slots %d %s\n", st, dqmc_last_error()); return 1; }
        slot_req[c] = next; left[c] = sweeps[next]; ++next;
      }
    }
  }
  dqmc_destroy(b);
  std::free(w);
  std::fprintf(stderr, "served %d requests in %d ticks\n", n_req, ticks);
  // alone
  int bad = 0;
  for (int r = 0; r < n_req; ++r) {
    char* w1 = nullptr;
    dqmc_batch* b1 = nullptr;
    run_batch(1, &seeds[r], &w1, &b1);
    dqmc_sweep(b1, sweeps[r], nullptr);
    Result a = take(b1, 1, 0);
    dqmc_destroy(b1);
    std::free(w1);
    const Result& s = served[r];
    const bool same = a.fields == s.fields && a.obs.double_occ == s.obs.double_occ &&
                      a.obs.kinetic == s.obs.kinetic && a.obs.logdet_up == s.obs.logdet_up &&
                      a.obs.accepted == s.obs.accepted && a.obs.max_drift == s.obs.max_drift;
    std::printf("request %d sweeps %d: %s (docc %.15g vs %.15g, drift %.3g, flags %d)\n", r, sweeps[r],
                same ? "same" : "DIFFERENT", s.obs.double_occ, a.obs.double_occ, s.obs.max_drift, s.obs.flags);
    bad += !same;
  }
  return bad ? 3 : 0;
}
