/*
 * dqmc.h -- C ABI of the MI355X batched DQMC sweep library (libdqmc.so).
 *
 * The library runs step 4 of the NIMC scheme (Alg. 1 of the paper): one short determinant QMC
 * Markov chain per starting Hubbard-Stratonovich (HS) configuration, many independent chains at
 * once, for the Hubbard model of eq. (3).  The problem is the one of supplement section I.2:
 * the inverse temperature beta = n_slices * dtau is cut into L_tau = n_slices Trotter slices,
 * the interaction is decoupled by a discrete HS field s_{i,l} = +-1 with cosh(nu) = e^{U dtau/2},
 * the slice propagator is B^sigma_l = e^{sigma nu Diag(s_l)} e^{-dtau T} and a field has weight
 * prod_sigma det[I + B^sigma(L_tau, 0)].  A sweep attempts one single-site flip at every
 * (slice, site) of the field (definition of a sweep in supplement section I.3).
 *
 * Conventions shared by every call:
 *   - Every function returns a dqmc_status; nothing throws or aborts across the ABI.
 *   - Device memory is owned by the caller (e.g. torch tensors); the library never calls
 *     hipMalloc or hipFree.  It owns only the opaque host-side dqmc_batch handle.
 *   - "stream" is a hipStream_t (NULL = the default stream).  Calls enqueue work on it and
 *     return; only dqmc_init_chains and dqmc_measure wait for their own work (to report input
 *     errors and numerical flags).  A handle is used from one stream at a time and is not
 *     thread-safe.
 *   - Matrices are row-major.  Sites are 0 .. N-1, slices l = 1 .. L_tau are stored at
 *     index l-1 of the field, spins are index 0 (up, sigma = +1) and 1 (down, sigma = -1).
 *   - dqmc_last_error() returns a thread-local message describing the last failure.
 */
#ifndef DQMC_H
#define DQMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DQMC_OK = 0,
  DQMC_EINVAL = -1,   /* bad shape or parameter, or a field value other than +-1 */
  DQMC_ENOMEM = -2,   /* the caller's workspace is smaller than dqmc_workspace_bytes */
  DQMC_EDEVICE = -3,  /* a HIP runtime error (message in dqmc_last_error) */
  DQMC_ENUMERIC = -4, /* at least one chain raised a numerical flag (see dqmc_obs.flags) */
  DQMC_EBUSY = -5     /* reserved: the handle is in use */
} dqmc_status;

typedef enum {
  DQMC_FP64 = 0,       /* everything in FP64 */
  DQMC_FP32_WRAP = 1   /* wraps and delayed updates in FP32 (MFMA); QR/UDT stabilisation,
                          fresh Green's functions and every acceptance ratio stay in FP64 */
} dqmc_precision;

/* Per-chain flags (dqmc_obs.flags) */
#define DQMC_FLAG_NONFINITE 1   /* a ratio or a Green's function went non-finite */
#define DQMC_FLAG_NEGATIVE 2    /* R < 0 (cannot happen at half filling on a bipartite lattice) */
#define DQMC_FLAG_DRIFT 4       /* |G_wrapped - G_fresh| exceeded dqmc_model.drift_limit */
#define DQMC_FLAG_SINGULAR 8    /* a zero pivot in QR or LU */

/* The model (supplement section I.2).  All values are read during dqmc_init_chains. */
typedef struct {
  int32_t n_sites;          /* N >= 1 */
  const double* hopping;    /* HOST, N*N row-major symmetric T (T_ij = -t per bond); copied */
  double U;                 /* on-site repulsion (>= 0) */
  double mu;                /* chemical potential: T -> T - mu I (0 = half filling) */
  double dtau;              /* Trotter step; beta = n_slices * dtau */
  int32_t n_slices;         /* L_tau >= 1 */
  int32_t stab_every;       /* FP64: slices between QR/UDT stabilisations (fresh G); >= 1 */
  int32_t refresh_every;    /* FP32_WRAP: slices between FP64 fresh-G refreshes (0 = stab_every).
                               The refresh points are also the stabilisation points. */
  int32_t delay_rank;       /* k: sites per delayed-update block (0 = library default: 16, 32 from
                               N = 128 on) */
  int32_t precision;        /* dqmc_precision */
  int32_t qr_blocked;       /* 0: column-pivoted Householder QR in every stabilisation (default).
                               1: for 64 < N <= 512, blocked Householder QR with the columns
                               pre-sorted by norm once (MFMA trailing updates; much faster at
                               large N).  It reproduces the pivoted G only while the products are
                               mildly graded; enable it for a model only after checking that on
                               fixed fields (the autotuner does).  Ignored elsewhere. */
  int32_t sweep_mode;       /* 0: every sweep an up sweep (slices 1 .. L_tau), right UDT stack
                               rebuilt per sweep.  Bit 0: odd global sweeps run down (attempt
                               slice l at G(l), then G(l-1) = B_l^{-1} G(l) B_l), each direction
                               reusing the UDT stack the other one left.  Bit 1: the equal-time
                               estimators are also taken after every slice (dqmc_obs.slice_*).
                               Nonzero modes run in the workspace kernels at any N. */
  double drift_limit;       /* DQMC_FLAG_DRIFT is raised when max|G_wrapped - G_fresh| at a
                               stabilisation point exceeds this (0 = default: 1e-3 in FP64, 1e-5 in
                               FP32_WRAP, the bound its Green's functions are meant to keep) */
} dqmc_model;

/* Observables of one chain, written by dqmc_measure (device memory, one per chain).  The
 * estimators use the equal-time Green's function G(0) = G(L_tau) that the last stabilisation
 * of the last sweep left (a pure function of the current field). */
typedef struct {
  double double_occ;      /* (1/N) sum_i <n_i,up n_i,dn> */
  double density;         /* (1/N) sum_i <n_i,up + n_i,dn> */
  double kinetic;         /* (1/N) sum_sigma sum_ij T_ij <c+_i c_j> */
  double logdet_up;       /* log|det(I + B^up(L_tau, 0))| */
  double logdet_dn;
  double max_drift;       /* max over stabilisations of max|G_wrapped - G_fresh| */
  double max_logdet_err;  /* max |log det from accumulated log R - fresh log det| */
  int64_t attempted;      /* flips attempted (sweeps * L_tau * N) */
  int64_t accepted;
  int64_t near_ties;      /* decisions with |u - R| < 1e-9 */
  int64_t sweeps_done;    /* global sweep counter of the chain (RNG counter, resume point) */
  int32_t flags;          /* DQMC_FLAG_* */
  int32_t reserved;
  double slice_double_occ; /* per-slice estimators (sweep_mode bit 1), averaged over every slice */
  double slice_kinetic;    /*   of every sweep since init; 0 without measurements */
  int64_t slice_meas;      /* number of slices measured */
} dqmc_obs;

typedef struct dqmc_batch dqmc_batch;   /* opaque host handle */
typedef struct dqmc_graph dqmc_graph;   /* opaque recorded sweep of several batches */

/* Device bytes one chain needs (the admission unit of a memory budget). */
size_t dqmc_chain_bytes(const dqmc_model* m);

/* Device workspace for n_chains chains of model m (shared constants + per-chain state). */
size_t dqmc_workspace_bytes(const dqmc_model* m, int32_t n_chains);

/* Create n_chains chains and compute their initial Green's functions G(0).
 *   fields: DEVICE int8 [n_chains][n_slices][N] of +-1 (copied into the workspace), or NULL to
 *           draw each chain's field from its seed (Philox4x64-10, key (seed, 0): element
 *           e = l*N + i is +1 iff the low bit of raw output word e is 1).
 *   seeds:  HOST uint64 [n_chains]; the key of each chain's acceptance random numbers.
 *   workspace: DEVICE, at least dqmc_workspace_bytes(m, n_chains) bytes, 256-byte aligned,
 *           owned by the caller and kept alive until dqmc_destroy.
 * Waits for its own work; returns EINVAL for a field value other than +-1. */
dqmc_status dqmc_init_chains(dqmc_batch** out, const dqmc_model* m, int32_t n_chains,
                             const int8_t* fields, const uint64_t* seeds, void* workspace,
                             size_t ws_bytes, void* stream);

/* Run n_sweeps Metropolis sweeps on every chain of the batch (one persistent launch). */
dqmc_status dqmc_sweep(dqmc_batch* b, int32_t n_sweeps, void* stream);

/* Per-sweep series (chain diagnostics: autocorrelation, convergence from the starting fields).
 * Runs n_sweeps sweeps exactly as dqmc_sweep and, after each sweep s, writes every chain c's
 * equal-time estimators at that sweep's fresh G(0) = G(L_tau) into
 * series[(s * n_chains + c) * DQMC_SERIES_WIDTH + k]: k = 0 double occupancy, 1 density,
 * 2 kinetic energy (the values dqmc_measure would return after that sweep), 3 the structure
 * factor of the form factor `form` (the value dqmc_spin_structure would return; 0 if form is
 * NULL).  No host synchronisation between sweeps.
 *   form:   DEVICE double [N] or NULL.   series: DEVICE double [n_sweeps][n_chains][4].
 * The NIMC analysis of the paper (main text Fig. 3, supplement eq. (5)) is built on such series
 * of observables against the sweep index. */
#define DQMC_SERIES_WIDTH 4
dqmc_status dqmc_sweep_series(dqmc_batch* b, int32_t n_sweeps, const double* form, double* series,
                              void* stream);

/* Sweep several batches (e.g. different lattice sizes) together: one launch per batch, all
 * enqueued before any waits, the batches overlapping on the device through forked streams. */
dqmc_status dqmc_sweep_multi(dqmc_batch* const* bs, const int32_t* n_sweeps, int32_t n,
                             void* stream);

/* Re-initialise chains slots[0 .. n_slots-1] of an existing batch (continuous batching: a chain
 * slot freed by a finished request takes a new one).  Each listed chain gets a new field and seed
 * exactly as dqmc_init_chains would give chain i of a new batch (its result does not depend on
 * the batch it runs in) and its counters restart at zero; other chains are untouched.
 *   slots:  HOST int32 [n_slots], distinct, in [0, n_chains).
 *   fields: DEVICE int8 [n_slots][n_slices][N] of +-1, or NULL to draw them from the seeds.
 *   seeds:  HOST uint64 [n_slots].
 * Waits for its own work; returns EINVAL for a bad slot list or field value.  Must not overlap
 * a sweep of the same batch (order the two on one stream). */
dqmc_status dqmc_init_slots(dqmc_batch* b, const int32_t* slots, int32_t n_slots,
                            const int8_t* fields, const uint64_t* seeds, void* stream);

/* One persistent launch in which chain c runs counts[c] sweeps (0 = idle this launch).
 *   counts: DEVICE int32 [n_chains], read by the kernel when it runs (the caller keeps it
 *           alive and unchanged until the launch has completed on the stream). */
dqmc_status dqmc_sweep_counts(dqmc_batch* b, const int32_t* counts, void* stream);

/* Record n_sweeps[i] sweeps of every batch bs[i] as one HIP graph of independent kernel nodes
 * (batches of different lattices run side by side).  Each dqmc_graph_launch replays the
 * recording and advances the chains by those sweeps, with the same results as the same calls
 * of dqmc_sweep_multi.  The batches must outlive the graph; n >= 1. */
dqmc_status dqmc_graph_create(dqmc_graph** out, dqmc_batch* const* bs, const int32_t* n_sweeps,
                              int32_t n);
dqmc_status dqmc_graph_launch(dqmc_graph* g, void* stream);
dqmc_status dqmc_graph_destroy(dqmc_graph* g);

/* Per-chain observables into obs (DEVICE [n_chains]); if green != NULL also both spins' G(0)
 * into green (DEVICE double [n_chains][2][N][N]).  Waits; returns ENUMERIC if any flag is set
 * (the outputs are written regardless). */
dqmc_status dqmc_measure(dqmc_batch* b, dqmc_obs* obs, double* green, void* stream);

/* Magnetic structure factor of every chain at G(0) (main text eq. (4): S(Q) = (1/N) sum_ij
 * e^{-iQ.(r_i - r_j)} <s^z_i s^z_j>, s^z = (n_up - n_dn)/2), for a real form factor f:
 * out[c] = (1/N) sum_ij f_i f_j <s^z_i s^z_j>, evaluated by Wick's theorem at chain c's field.
 * Phases +-1 (a sublattice sign) give S(Q) directly; a complex phase e^{iQ.r} is the sum of the
 * results for f = cos(Q.r) and f = sin(Q.r).
 *   form: DEVICE double [N].   out: DEVICE double [n_chains].
 * Asynchronous on the stream; same G(0) as dqmc_measure. */
dqmc_status dqmc_spin_structure(dqmc_batch* b, const double* form, double* out, void* stream);

/* Current fields into out (DEVICE int8 [n_chains][n_slices][N]). */
dqmc_status dqmc_get_fields(dqmc_batch* b, int8_t* out, void* stream);

/* Release the host handle (the workspace stays the caller's). */
dqmc_status dqmc_destroy(dqmc_batch* b);

const char* dqmc_last_error(void);

/* A HIP stream of the caller's own, for batches that run side by side (one resident batch per
 * model in a serving loop): non-blocking with respect to the null stream, default priority,
 * on the current device.  The HIP runtime maps streams onto a few hardware queues per process
 * (GPU_MAX_HW_QUEUES) and kernels of streams that share a queue run one after the other; streams
 * created together are spread over the queues by the runtime, unlike pooled streams created
 * earlier for other uses.  out receives the hipStream_t.  dqmc_stream_destroy waits for the
 * stream's work, then destroys it; the caller first releases everything that still refers to
 * the stream (events recorded on it, allocator records of host buffers copied on it). */
dqmc_status dqmc_stream_create(void** out);
dqmc_status dqmc_stream_destroy(void* stream);

/* For callers that cannot allocate device memory (code that must not call hipMalloc: under HIP
 * graph capture, in tight serving loops, in harnesses that forbid it): the sequence
 * dqmc_init_chains -> dqmc_sweep(n_sweeps) -> dqmc_measure (and dqmc_get_fields) in one call, on
 * the same kernels and with the same results, the chains' state held in a static device array of
 * the library (DQMC_STATIC_BYTES on each GPU it runs on, kept until the process ends) instead of
 * a caller workspace, and no host handle.  It allocates no device or host memory.
 *   m, n_chains, fields, seeds: as dqmc_init_chains.   n_sweeps >= 0.
 *   obs:        DEVICE dqmc_obs [n_chains], required.
 *   green:      DEVICE double [n_chains][2][N][N] or NULL (both spins' G(0) after the sweeps).
 *   fields_out: DEVICE int8 [n_chains][n_slices][N] or NULL (the fields after the sweeps).
 * Returns EINVAL when dqmc_workspace_bytes(m, n_chains) exceeds DQMC_STATIC_BYTES (and for the
 * reasons dqmc_init_chains gives), ENUMERIC as dqmc_measure (outputs written regardless).  Waits
 * for its work.  All calls on one GPU share that GPU's array, which keeps the last call's
 * contents (each call initialises what it uses): calls that overlap on one GPU, from several
 * host threads or on streams not ordered with each other, race and must be serialised. */
#define DQMC_STATIC_BYTES ((size_t)64 << 20)
dqmc_status dqmc_run_static(const dqmc_model* m, int32_t n_chains, const int8_t* fields,
                            const uint64_t* seeds, int32_t n_sweeps, dqmc_obs* obs, double* green,
                            int8_t* fields_out, void* stream);

/* Numbers the library chose: site-block size k, stabilisation interval, LDS bytes of the sweep
 * kernel, and the sweep kernel variant (0 = generic with LDS-resident Green's functions,
 * 1 = generic with Green's functions in the workspace, 2 = the N <= 64 register/LDS path). */
dqmc_status dqmc_batch_info(const dqmc_batch* b, int32_t* k, int32_t* stab, int32_t* lds_bytes,
                            int32_t* variant);

/* ---- fixed-field probes for parity tests: no acceptance, no change of fields or G(0) ---- */

/* Fresh G^sigma(slice) = [I + B(slice,0) B(L_tau,slice)]^{-1} of every chain's current field,
 * then n_wraps wraps G <- B_l G B_l^{-1} (l = slice+1 .. slice+n_wraps) in the batch's wrap
 * precision, or for n_wraps < 0 the down sweeps' unwraps G <- B_l^{-1} G B_l (l = slice,
 * slice-1, .., slice+n_wraps+1).  out: DEVICE double [n_chains][2][N][N].
 * 0 <= slice <= L_tau, 0 <= slice + n_wraps <= L_tau. */
dqmc_status dqmc_debug_green(dqmc_batch* b, int32_t slice, int32_t n_wraps, double* out,
                             void* stream);

/* Ratios R^sigma_i = 1 + Delta^sigma_i (1 - G^sigma_ii(slice)) for flipping s_{i,slice} alone,
 * from the fresh G(slice).  out: DEVICE double [n_chains][2][N].  1 <= slice <= L_tau. */
dqmc_status dqmc_debug_ratios(dqmc_batch* b, int32_t slice, double* out, void* stream);

/* The propagators e^{-dtau (T - mu)} and e^{+dtau (T - mu)} the batch computed on the device.
 * out: DEVICE double [2][N][N]. */
dqmc_status dqmc_debug_propagators(dqmc_batch* b, double* out, void* stream);

/* Wall-clock ticks (100 MHz) each chain's workgroup spent per phase of its sweeps since init:
 * [0] right stack, [1] wraps, [2] Metropolis decisions, [3] delayed-update panels, [4] rank-m
 * flushes, [5] left UDT, [6] fresh G, [7] whole sweeps; finer split of the stabilisation work
 * (N <= 64 path): [8] B-chunk products, [9] QR factorisation, [10] forming Q, [11] T products,
 * [12] fresh-G products, [13] Gauss-Jordan, [14] fresh-G output product, [15] parking G.
 * out: DEVICE int64 [n_chains][16]. */
dqmc_status dqmc_debug_phase_ticks(dqmc_batch* b, int64_t* out, void* stream);

/* Raw Philox4x64-10 blocks of the device generator: for counters (c0 + j, c1, c2, c3),
 * j = 0 .. n_blocks-1, key (k0, k1), the four words into out (DEVICE uint64 [n_blocks][4]). */
dqmc_status dqmc_debug_philox(uint64_t k0, uint64_t k1, uint64_t c0, uint64_t c1, uint64_t c2,
                              uint64_t c3, int32_t n_blocks, uint64_t* out, void* stream);

/* One 16x16x4 matrix-core product per precision: A (16x4), B (4x16) row-major DEVICE inputs,
 * C = A B written row-major into out64 (double[256]) and out32 (float[256]); checks the lane
 * layout the library assumes for each instruction. */
dqmc_status dqmc_debug_mfma(const double* a64, const double* b64, double* out64,
                            const float* a32, const float* b32, float* out32, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* DQMC_H */
