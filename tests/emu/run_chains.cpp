// Test-only: the library's C ABI on the host emulation (emu_hip.h).  Reads a model, fields and
// seeds from DIR (header.txt, hop.bin, fields.bin, seeds.bin), runs dqmc_init_chains, n_sweeps
// one-sweep dqmc_sweep calls, dqmc_measure and dqmc_get_fields, and writes obs.bin, green.bin and
// fields_out.bin to DIR.  The workspace is one exact-size heap block, so AddressSanitizer sees
// any access past it; EMU_WS_FILL and EMU_LDS_FILL set the bytes the workspace and LDS start with.
// An optional second line of header.txt, "sweep_mode series static [qr_blocked=1]", selects the
// blocked stabilisation QR (dqmc_model.qr_blocked) and the sweep mode
// (dqmc_model.sweep_mode), dqmc_sweep_series in place of the one-sweep calls (series.bin,
// [n_sweeps][n_chains][4]), or the allocation-free dqmc_run_static in place of the whole
// sequence.  An optional third line "slice n_wraps" adds the fixed-field probe
// dqmc_debug_green(slice, n_wraps) right after the initialisation (probe.bin, [n_chains][2][N][N]).
// usage: run_chains DIR
#include "emu_hip.h"
#include "dqmc.h"
#include "dqmc_device.hpp"

void emu_call_kernel(const void* fn, void** params) {
  auto k = reinterpret_cast<void (*)(dqmc::KArgs)>(const_cast<void*>(fn));
  k(*reinterpret_cast<dqmc::KArgs*>(params[0]));
}

template <typename T>
static std::vector<T> readf(const std::string& p, size_t n) {
  std::vector<T> v(n);
  FILE* f = std::fopen(p.c_str(), "rb");
  if (!f || std::fread(v.data(), sizeof(T), n, f) != n) { std::fprintf(stderr, "read %s\n", p.c_str()); std::exit(2); }
  std::fclose(f);
  return v;
}
template <typename T>
static void writef(const std::string& p, const T* d, size_t n) {
  FILE* f = std::fopen(p.c_str(), "wb");
  std::fwrite(d, sizeof(T), n, f);
  std::fclose(f);
}

int main(int argc, char** argv) {
  std::string dir = argv[1];
  FILE* h = std::fopen((dir + "/header.txt").c_str(), "r");
  int n, L, stab, prec, refresh, k, n_chains, n_sweeps, have_fields;
  double drift, U, dtau;
  if (std::fscanf(h, "%d %d %d %d %d %d %lf %lf %lf %d %d %d", &n, &L, &stab, &prec, &refresh, &k, &drift, &U,
                  &dtau, &n_chains, &n_sweeps, &have_fields) != 12) return 2;
  int sweep_mode = 0, use_series = 0, use_static = 0, qr_blocked = 0;
  if (std::fscanf(h, "%d %d %d", &sweep_mode, &use_series, &use_static) != 3) sweep_mode = use_series = use_static = 0;
  if (std::fscanf(h, " qr_blocked=%d", &qr_blocked) != 1) qr_blocked = 0;
  int probe_slice = -1, probe_wraps = 0;
  if (std::fscanf(h, "%d %d", &probe_slice, &probe_wraps) != 2) probe_slice = -1;
  std::fclose(h);
  auto hop = readf<double>(dir + "/hop.bin", (size_t)n * n);
  auto seeds = readf<uint64_t>(dir + "/seeds.bin", n_chains);
  std::vector<int8_t> fields;
  if (have_fields) fields = readf<int8_t>(dir + "/fields.bin", (size_t)n_chains * L * n);
  dqmc_model m{};
  m.n_sites = n; m.hopping = hop.data(); m.U = U; m.mu = 0.0; m.dtau = dtau; m.n_slices = L;
  m.stab_every = stab; m.refresh_every = refresh; m.delay_rank = k;
  m.precision = prec ? DQMC_FP32_WRAP : DQMC_FP64; m.drift_limit = drift;
  m.sweep_mode = sweep_mode;
  m.qr_blocked = qr_blocked;
  if (use_static) {
    std::vector<dqmc_obs> obs(n_chains);
    std::vector<double> green((size_t)n_chains * 2 * n * n);
    std::vector<int8_t> fo((size_t)n_chains * L * n);
    int st = dqmc_run_static(&m, n_chains, have_fields ? fields.data() : nullptr, seeds.data(), n_sweeps,
                             obs.data(), green.data(), fo.data(), nullptr);
    std::fprintf(stderr, "run_static: %d %s\n", st, st ? dqmc_last_error() : "");
    if (st != DQMC_OK && st != DQMC_ENUMERIC) return 1;
    writef(dir + "/obs.bin", obs.data(), obs.size());
    writef(dir + "/green.bin", green.data(), green.size());
    writef(dir + "/fields_out.bin", fo.data(), fo.size());
    return 0;
  }
  const size_t ws = dqmc_workspace_bytes(&m, n_chains);
  char* w = (char*)std::aligned_alloc(256, (ws + 255) & ~(size_t)255);
  const char* wf = std::getenv("EMU_WS_FILL");
  std::memset(w, wf ? (int)std::strtol(wf, nullptr, 0) : 0xA5, ws);
  dqmc_batch* b = nullptr;
  int st = dqmc_init_chains(&b, &m, n_chains, have_fields ? fields.data() : nullptr, seeds.data(), w, ws, nullptr);
  std::fprintf(stderr, "init: %d %s\n", st, st ? dqmc_last_error() : "");
  if (st) return 1;
  int kk, ss, lds, var;
  dqmc_batch_info(b, &kk, &ss, &lds, &var);
  std::fprintf(stderr, "k %d stab %d lds %d variant %d\n", kk, ss, lds, var);
  if (probe_slice >= 0) {
    std::vector<double> g((size_t)n_chains * 2 * n * n);
    st = dqmc_debug_green(b, probe_slice, probe_wraps, g.data(), nullptr);
    std::fprintf(stderr, "debug_green(%d, %d): %d\n", probe_slice, probe_wraps, st);
    if (st) return 1;
    writef(dir + "/probe.bin", g.data(), g.size());
  }
  const long long m64_init = emu::mfma_issued(0), m32_init = emu::mfma_issued(1);
  if (use_series) {
    std::vector<double> series((size_t)n_sweeps * n_chains * DQMC_SERIES_WIDTH);
    st = dqmc_sweep_series(b, n_sweeps, nullptr, series.data(), nullptr);
    std::fprintf(stderr, "sweep_series: %d\n", st);
    writef(dir + "/series.bin", series.data(), series.size());
  } else {
    for (int s = 0; s < n_sweeps; ++s) {
      st = dqmc_sweep(b, 1, nullptr);
      std::fprintf(stderr, "sweep %d: %d\n", s, st);
    }
  }
  std::fprintf(stderr, "mfma issued in the sweeps: fp64 %lld fp32 %lld (init: fp64 %lld fp32 %lld)\n",
               emu::mfma_issued(0) - m64_init, emu::mfma_issued(1) - m32_init, m64_init, m32_init);
  std::vector<dqmc_obs> obs(n_chains);
  std::vector<double> green((size_t)n_chains * 2 * n * n);
  st = dqmc_measure(b, obs.data(), green.data(), nullptr);
  std::fprintf(stderr, "measure: %d %s\n", st, st ? dqmc_last_error() : "");
  std::vector<int8_t> fo((size_t)n_chains * L * n);
  dqmc_get_fields(b, fo.data(), nullptr);
  writef(dir + "/obs.bin", obs.data(), obs.size());
  writef(dir + "/green.bin", green.data(), green.size());
  writef(dir + "/fields_out.bin", fo.data(), fo.size());
  dqmc_destroy(b);
  std::free(w);
  return 0;
}
