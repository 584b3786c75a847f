"""Per-model choice of the knobs that change speed but not the method.

* Delay rank k (sites per delayed-update block).  Decisions do not depend on k, only rounding
  and speed do, so k is chosen by timing: each candidate runs a few sweeps of a small batch and
  the fastest wins.
* FP32-wrap refresh interval.  Wrapping G in FP32 loses accuracy geometrically with the number
  of wraps since the last FP64 refresh.  On fixed fields, the FP32-wrapped G after r wraps is
  compared with the FP64 fresh G of the same slice (max |dG| over sampled slices and chains);
  the largest r within the bound is chosen.  In sweeps the accepted flips amplify that error
  (the Sherman-Morrison update divides by the ratio), so `drift_interval` measures the drift the
  sweeps themselves see at the refresh points, from a short run per candidate.
* Stabilisation interval.  The drift max|G_wrapped - G_fresh| at the stabilisation points grows
  with the interval and with how strongly graded the B products are (U, beta).  `drift_interval`
  runs a few sweeps per candidate and keeps the largest interval whose drift stays within a bound.

* Stabilisation QR for N > 64.  The blocked QR with pre-sorted columns is much faster than the
  column-pivoted one but reproduces its Green's function only while the B products are mildly
  graded (strong coupling and low temperature spread the scales too far).  On fixed fields both
  are run and the blocked one is chosen when the fresh G of every sampled slice agrees within the
  bound.

Results are cached per model in a JSON file when a path is given.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Iterable, Optional, Sequence

import numpy as np

from . import dqmc


def _model_id(n_sites: int, n_slices: int, U: float, dtau: float, precision: str, extra="") -> str:
    return f"N{n_sites}_L{n_slices}_U{U:g}_dt{dtau:g}_{precision}{extra}"


class Autotuner:
    def __init__(self, cache_path: Optional[str] = None, device="cuda:0"):
        self.cache_path = cache_path
        self.device = device
        self.cache: Dict[str, dict] = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)

    def _save(self):
        if self.cache_path:
            tmp = self.cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)
            os.replace(tmp, self.cache_path)

    def delay_rank(self, hopping, U, dtau, n_slices, stab_every, precision="fp64", refresh_every=0,
                   candidates: Sequence[int] = (8, 16, 32), n_chains: int = 64, sweeps: int = 2,
                   seed: int = 0x7A11) -> dict:
        """Fastest delay rank among the candidates (the library clamps k to what its kernels
        support; candidates that map to the same k are timed once)."""
        T = np.asarray(hopping, dtype=np.float64)
        key = _model_id(T.shape[0], n_slices, U, dtau, precision, f"_r{refresh_every}_k")
        if key in self.cache:
            return self.cache[key]
        torch = dqmc._torch()
        seeds = np.arange(n_chains, dtype=np.uint64) + np.uint64(seed)
        timings, seen, eff_of = {}, {}, {}
        for k in candidates:
            m = dqmc.make_model(T, U, dtau, n_slices, stab_every, refresh_every=refresh_every,
                                delay_rank=k, precision=precision)
            b = dqmc.Batch(m, seeds, device=self.device)
            eff = b.delay_rank
            eff_of[k] = int(eff)
            if eff in seen:
                timings[k] = seen[eff]
                b.close()
                continue
            b.sweep(1)
            torch.cuda.synchronize(self.device)
            t0 = time.perf_counter()
            b.sweep(sweeps)
            torch.cuda.synchronize(self.device)
            dt = (time.perf_counter() - t0) / sweeps
            seen[eff] = dt
            timings[k] = dt
            b.close()
        best = min(timings, key=lambda k: timings[k])
        rec = {"delay_rank": int(best), "effective_delay_rank": eff_of[best],
               "seconds_per_sweep": {str(k): v for k, v in timings.items()},
               "effective": {str(k): v for k, v in eff_of.items()}}
        self.cache[key] = rec
        self._save()
        return rec

    def refresh_interval(self, hopping, U, dtau, n_slices, fields, seeds, bound: float = 1e-5,
                         candidates: Iterable[int] = (2, 3, 4, 5, 6, 8, 10),
                         slices: Optional[Sequence[int]] = None, stab_every: int = 10) -> dict:
        """Largest FP32-wrap refresh interval whose wrap error stays within `bound` on the given
        fixed fields (int8 [chains][n_slices][N]); the error of r wraps from slice l is
        max |G_fp32(l -> l + r) - G_fp64_fresh(l + r)| over chains and sampled slices."""
        T = np.asarray(hopping, dtype=np.float64)
        key = _model_id(T.shape[0], n_slices, U, dtau, "fp32_wrap", f"_b{bound:g}_refresh")
        if key in self.cache:
            return self.cache[key]
        cands = sorted(int(r) for r in candidates if 1 <= int(r) <= n_slices)
        if slices is None:
            slices = sorted({0, n_slices // 3, (2 * n_slices) // 3})
        # fresh G from UDT chains stabilised every stab_every slices in both precisions; the
        # FP32 batch only differs in how it wraps
        m64 = dqmc.make_model(T, U, dtau, n_slices, stab_every, precision="fp64")
        m32 = dqmc.make_model(T, U, dtau, n_slices, stab_every, refresh_every=stab_every,
                              precision="fp32_wrap")
        b64 = dqmc.Batch(m64, seeds, fields, device=self.device)
        b32 = dqmc.Batch(m32, seeds, fields, device=self.device)
        errs = {}
        for r in cands:
            e = 0.0
            for l in slices:
                if l + r > n_slices:
                    continue
                g32 = b32.debug_green(l, r)
                g64 = b64.debug_green(l + r, 0)
                e = max(e, float((g32 - g64).abs().max().item()))
            errs[r] = e
        b64.close()
        b32.close()
        best = 1
        for r in cands:              # the longest interval whose shorter ones all pass too
            if errs[r] > bound:
                break
            best = r
        rec = {"refresh_every": int(best), "bound": bound, "max_abs_dG": {str(r): v for r, v in errs.items()}}
        self.cache[key] = rec
        self._save()
        return rec

    def drift_interval(self, hopping, U, dtau, n_slices, fields, seeds, bound: float,
                       candidates: Sequence[int] = (10, 8, 5, 4, 2), precision: str = "fp64",
                       sweeps: int = 2, stab_every: int = 10) -> dict:
        """Largest interval (stabilisation interval in FP64, refresh interval in FP32_WRAP) whose
        drift at the stabilisation points, max over the chains of a run of `sweeps` sweeps from the
        given fields, stays within `bound`.  Candidates are tried from the largest down; the
        result says whether any met the bound (`meets_bound`) and keeps the drift of each."""
        T = np.asarray(hopping, dtype=np.float64)
        key = _model_id(T.shape[0], n_slices, U, dtau, precision,
                        f"_b{bound:g}_s{sweeps}_c{len(seeds)}_drift")
        if key in self.cache:
            return self.cache[key]
        cands = sorted({int(r) for r in candidates if 1 <= int(r) <= n_slices}, reverse=True)
        drift, secs, chosen = {}, {}, None
        torch = dqmc._torch()
        for r in cands:
            if precision == "fp32_wrap":
                m = dqmc.make_model(T, U, dtau, n_slices, stab_every, refresh_every=r,
                                    precision=precision, drift_limit=1.0)
            else:
                m = dqmc.make_model(T, U, dtau, n_slices, r, precision=precision, drift_limit=1.0)
            b = dqmc.Batch(m, seeds, fields, device=self.device)
            torch.cuda.synchronize(self.device)
            t0 = time.perf_counter()
            b.sweep(sweeps)
            torch.cuda.synchronize(self.device)
            secs[r] = (time.perf_counter() - t0) / sweeps
            o = b.measure()
            b.close()
            drift[r] = float(o["max_drift"].max())
            if drift[r] <= bound:
                chosen = r
                break
        rec = {"interval": int(chosen if chosen is not None else cands[-1]),
               "meets_bound": chosen is not None, "bound": bound, "precision": precision,
               "sweeps": sweeps, "chains": int(len(seeds)),
               "max_drift": {str(r): v for r, v in drift.items()},
               "seconds_per_sweep": {str(r): v for r, v in secs.items()}}
        self.cache[key] = rec
        self._save()
        return rec

    def qr_method(self, hopping, U, dtau, n_slices, fields, seeds, stab_every: int = 10,
                  bound: float = 1e-11, slices: Optional[Sequence[int]] = None) -> dict:
        """Use the blocked QR (qr_blocked = 1) when its fresh G matches the column-pivoted one
        within `bound` (max |dG| over chains and sampled slices) on the given fixed fields."""
        T = np.asarray(hopping, dtype=np.float64)
        N = T.shape[0]
        key = _model_id(N, n_slices, U, dtau, "fp64", f"_s{stab_every}_b{bound:g}_qr")
        if key in self.cache:
            return self.cache[key]
        if N <= 64 or N > 512:
            rec = {"qr_blocked": False, "max_abs_dG": None, "reason": "blocked QR not used at this N"}
        else:
            if slices is None:
                slices = sorted({0, n_slices // 2, n_slices})
            ms = [dqmc.make_model(T, U, dtau, n_slices, stab_every, qr_blocked=qb) for qb in (False, True)]
            bs = [dqmc.Batch(m, seeds, fields, device=self.device) for m in ms]
            err = 0.0
            for l in slices:
                g0 = bs[0].debug_green(int(l), 0)
                g1 = bs[1].debug_green(int(l), 0)
                err = max(err, float((g0 - g1).abs().max().item()))
            for b in bs:
                b.close()
            rec = {"qr_blocked": bool(err <= bound), "max_abs_dG": err, "bound": bound}
        self.cache[key] = rec
        self._save()
        return rec
