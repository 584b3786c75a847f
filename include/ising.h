/* Batched Metropolis sweeps of the square-lattice Ising model on one MI355X.
 *
 * The paper's first benchmark (main text eq. (1), H = -J sum_<ij> s_i s_j on a periodic L x L
 * lattice; supplement section I.1) is sampled by local Metropolis updates, one attempt per spin
 * and sweep (supplement section I.3); Table 1 reports |M| = (1/N)|sum_i s_i| and E = <H>/N.
 * This library runs many independent chains side by side, one workgroup per chain, with the
 * lattice resident in LDS for the whole launch.
 *
 * Sweep: checkerboard order (every site with x + y even, then the odd ones; sites of one colour
 * do not interact, so each colour is one parallel step and the sweep equals a sequential
 * one-attempt-per-spin sweep in that order).  A flip of s at (x, y) with neighbour sum h changes
 * the energy by dE = 2 J s h and is accepted iff u < min(1, exp(-dE / T)), u uniform in [0, 1):
 * the top 53 bits of word q of Philox4x64-10 with key (seed, 0) and counter (b, 0, global sweep,
 * 2), for row-major site 4 b + q.  Initial spins drawn from the seed follow the DQMC field rule
 * (site e is +1 iff the low bit of raw word e of counter blocks (e / 4, 0, 0, 0) is 1).
 * A chain's trajectory is a pure function of its seed, its initial spins and its sweep counter.
 *
 * Observables are exact integers: M = sum_i s_i and the bond sum B = sum_i s_i (s_right +
 * s_down), so E = -J B and |M|/N, E/N follow on the host without rounding in the sums.
 *
 * Every call returns a dqmc_status (see dqmc.h); dqmc_last_error() gives the message.
 */
#ifndef ISING_H
#define ISING_H

#include <stddef.h>
#include <stdint.h>

#include "dqmc.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Per-chain counters (device memory, written by ising_stats).  The sums run over the sweeps
 * that were run with measure != 0. */
typedef struct {
  int64_t sweeps_done;  /* global sweep counter (RNG counter, resume point) */
  int64_t accepted;     /* accepted flips over all sweeps */
  int64_t n_meas;       /* measured sweeps */
  int64_t sum_abs_m;    /* sum of |M| after each measured sweep */
  int64_t sum_m2;       /* sum of M^2 */
  int64_t sum_bond;     /* sum of B (E = -J B) */
  int64_t sum_bond2;    /* sum of B^2 */
  int64_t reserved;
} ising_obs;

typedef struct ising_batch ising_batch;   /* opaque host handle */

/* Device workspace for n_chains chains of an L x L lattice (spins, counters, seeds). */
size_t ising_workspace_bytes(int32_t L, int32_t n_chains);

/* Create n_chains chains.
 *   L: even, 2 <= L <= 64.   J: coupling (any sign, finite).   T: temperature > 0.
 *   spins: DEVICE int8 [n_chains][L*L] of +-1 (row-major, copied), or NULL to draw them.
 *   seeds: HOST uint64 [n_chains].
 *   workspace: DEVICE, >= ising_workspace_bytes(L, n_chains) bytes, 256-byte aligned, owned by
 *              the caller and kept alive until ising_destroy.
 * Waits for its own work; EINVAL for a bad size, temperature or spin value, ENOMEM for a small
 * workspace. */
dqmc_status ising_init(ising_batch** out, int32_t L, double J, double T, int32_t n_chains,
                       const int8_t* spins, const uint64_t* seeds, void* workspace,
                       size_t ws_bytes, void* stream);

/* Run n_sweeps sweeps of every chain in one launch.  measure != 0 adds every sweep's M and B to
 * the chain's sums.  series (DEVICE int32 [n_chains][n_sweeps][2], or NULL) receives (M, B)
 * after each sweep.  Asynchronous on the stream. */
dqmc_status ising_sweep(ising_batch* b, int32_t n_sweeps, int32_t measure, int32_t* series,
                        void* stream);

/* Per-chain counters into out (DEVICE ising_obs [n_chains]).  Asynchronous. */
dqmc_status ising_stats(ising_batch* b, ising_obs* out, void* stream);

/* Current spins into out (DEVICE int8 [n_chains][L*L]).  Asynchronous. */
dqmc_status ising_get_spins(ising_batch* b, int8_t* out, void* stream);

/* Frees the host handle (the workspace is the caller's). */
dqmc_status ising_destroy(ising_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* ISING_H */
