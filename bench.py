"""Throughput of batched DQMC sweeps on one MI355X: HS-field updates per second.

Workload: 256 independent chains of the half-filled Hubbard model on an 8x8 periodic square
lattice, t=1, U=4, beta=4, dtau=0.1 (40 slices), stabilisation every 10 slices, each chain started
from a seeded uniform +-1 field (synthetic stand-in for network-generated configurations).
A step is one sweep of every chain (one persistent kernel launch); one update is one attempted
single-site flip, so a step performs 256 * 40 * 64 = 655,360 updates.

Prints one JSON line.  `value` is the FP64 throughput; the FP32-wrap form, its max|dG| against
the FP64 Green's function at every refresh point, the roofline of the dominant kernel and the
CPU oracle on a bounded sample ride along in the same line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# The serving leg keeps one stream per resident pool (nine at a time).  HIP maps streams onto
# GPU_MAX_HW_QUEUES hardware queues per process (4 by default), and pools whose streams share a
# queue run one after the other.  Ask for at least 16; the legs that use one stream occupy one
# queue either way.  The runtime reads it when it starts, so it is set before anything else.
SERVING_HW_QUEUES = 16
if not os.environ.get("GPU_MAX_HW_QUEUES", "").isdigit() or \
        int(os.environ["GPU_MAX_HW_QUEUES"]) < SERVING_HW_QUEUES:
    os.environ["GPU_MAX_HW_QUEUES"] = str(SERVING_HW_QUEUES)

import dqmc_inputs as di  # noqa: E402

PEAK_FP64_MFMA = 78.6e12     # MI355X dense FP64 matrix, FLOP/s
PEAK_FP32_MFMA = 157.3e12    # MI355X dense FP32 matrix, FLOP/s
WORKLOAD = "square8x8_U4_b4"
# the sources that define the headline kernel (fast_sweep_kernel<64, double, 16>)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2106_00712_amd", "csrc", f)
                  for f in ("dqmc_device.hpp", "dqmc_fast.hpp", "dqmc_stab.hpp", "philox.hpp",
                            "k_fast.hpp", "k_fast_f64_np64.hip")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fast_sweep_kernel_square8x8.json")


def algorithmic_flops(N: int, L: int, n_s: int, acc: float) -> dict:
    """Algorithmic FLOP of one sweep of one chain (both spins), by step of the method.

    wrap         2 spins x 2 products x 2N^3 per slice                         = 8 L N^3
    update       4 N^2 per accepted flip (rank-1 G update, both spins)        = 4 a L N^3
    chain        left B-chunk products 2N^3 per slice and spin, right stack    = 4 L N^3 + 4 (L - n_s) N^3
    qr           Householder QR (4/3 N^3) + explicit Q (4/3 N^3) + T update (N^3), 2 J - 1 per spin
    fresh_g      U_L^T U_R and T_L T_R^T (4N^3), LU + solve (8/3 N^3), U_R Z (2N^3), J per spin
    with J = ceil(L / n_s) stabilisation points and a the acceptance rate.
    """
    J = -(-L // n_s)
    n3 = float(N) ** 3
    parts = {
        "wrap": 8.0 * L * n3,
        "update": 4.0 * acc * L * n3,
        "chain": 4.0 * L * n3 + 4.0 * (L - n_s) * n3,
        "qr": 2.0 * (2 * J - 1) * (4.0 / 3 + 4.0 / 3 + 1.0) * n3,
        "fresh_g": 2.0 * J * (4.0 + 8.0 / 3 + 2.0) * n3,
    }
    parts["total"] = sum(parts.values())
    return parts


def row_rooflines(fl: dict, share: dict, t_launch: float, n_chains: int, peak: float) -> dict:
    """Each step of the path against the FP64 matrix peak: its algorithmic FLOP (per chain-sweep,
    times the chains of one launch) over the time the in-kernel phase counters give it."""
    groups = {
        "wrap": (["wrap"], ["wrap"]),
        "ratio_accept": ([], ["decide"]),
        "update": (["update"], ["panel", "flush"]),
        "stabilisation": (["chain", "qr", "fresh_g"], ["right_stack", "left_udt", "fresh_g"]),
    }
    out = {}
    for row, (fparts, phases) in groups.items():
        t = sum(share.get(p, 0.0) for p in phases) * t_launch
        f = sum(fl[p] for p in fparts) * n_chains
        out[row] = {"ms": t * 1e3, "share": t / t_launch if t_launch else None,
                    "tflops": (f / t / 1e12) if (t > 0 and f > 0) else None,
                    "frac": (f / t / peak) if (t > 0 and f > 0) else None}
    return out


def kernel_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def load_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter runs, if still current."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sha") != kernel_sha():
        return None
    return rec.get("bytes_per_launch")


def choose_qr(w, mode: str) -> bool:
    """Stabilisation QR of the N > 64 kernels: 'pivoted', 'blocked', or 'auto' (the autotuner's
    accuracy check on two chains' fixed fields)."""
    if mode != "auto":
        return mode == "blocked"
    from paper_2106_00712_amd.autotune import Autotuner
    return Autotuner().qr_method(w.hopping(), w.U, w.dtau, w.n_slices, w.fields(2), w.seeds(2),
                                 w.stab_every)["qr_blocked"]


def run_gpu(w, precision: str, steps: int, warmup: int, delay_rank: int, refresh: int,
            qr_blocked: bool = False, sweep_mode: int = 0, stab: int = 0):
    import torch
    from paper_2106_00712_amd import dqmc

    m = dqmc.make_model(w.hopping(), w.U, w.dtau, w.n_slices, stab or w.stab_every, delay_rank=delay_rank,
                        precision=precision, refresh_every=refresh, qr_blocked=qr_blocked,
                        sweep_mode=sweep_mode)
    fields = torch.as_tensor(w.fields()).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = dqmc.Batch(m, w.seeds(), fields)
    torch.cuda.synchronize()
    init_ms = (time.perf_counter() - t0) * 1e3
    for _ in range(warmup):
        b.sweep(1)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(steps):
        b.sweep(1)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_launch_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    obs = b.measure()
    ph = b.phase_seconds().mean(axis=0)
    tot = ph[7]
    share = {k: float(v / tot) for i, (k, v) in enumerate(zip(b.PHASES, ph)) if i != 7 and v > 0} \
        if tot > 0 else {}
    return dict(batch=b, wall=wall, per_launch_ms=per_launch_ms, init_ms=init_ms, obs=obs,
                phase_share=share)


def run_serving(rate: float, n_req: int, Ls, precision: str, capacity: int, tick: int,
                refresh: int, seed: int = 4, progress: bool = False):
    """Continuous batching of a Poisson stream of chain requests at `rate` req/s offered (lattice
    L x L with L uniform over `Ls`, beta and sweep count drawn as in the serving workload), warm
    pools for every model of the mix."""
    from paper_2106_00712_amd.serving import GpuExecutor, Request, Server, latency_stats
    reqs = di.serving_requests(n_req, rate, seed, Ls=tuple(Ls))
    ex = GpuExecutor(di.square_hopping, U=4.0, dtau=0.1, stab_every=10,
                     refresh_every=refresh if precision == "fp32_wrap" else 0)
    srv = Server(ex, hbm_budget=96 << 30, tick_sweeps=tick, pool_capacity=capacity,
                 precision=precision)
    srv.warm([(L, b) for L in Ls for b in di.SERVING_BETA])
    # the arrival times are re-based so that the first request arrives at t = 0
    t_first = reqs[0]["arrival"]
    rq = [Request(d["id"], d["L"], d["beta"], d["sweeps"], d["seed"], d["arrival"] - t_first)
          for d in reqs]
    t0 = time.perf_counter()
    try:
        res = srv.run(rq, progress=(lambda msg: print(f"serving {precision} {rate:g} req/s: {msg}",
                                                      file=sys.stderr, flush=True)) if progress else None)
        wall = time.perf_counter() - t0
    finally:
        srv.close()
    st = latency_stats(res)
    span = rq[-1].arrival if len(rq) > 1 else 0.0
    wait = [r.admitted - r.arrival for r in res]
    service = [r.finished - r.admitted for r in res]
    flagged = sum(1 for r in res if int(r.obs["flags"]))
    return {"rate_req_per_s": rate, "measured_arrival_rate_req_per_s": (len(rq) - 1) / span if span > 0 else None,
            "requests": len(res), "p50_s": st["p50_s"], "p99_s": st["p99_s"],
            "mean_s": st["mean_s"], "wait_p50_s": float(np.median(wait)) if wait else None,
            "wait_p99_s": float(np.percentile(wait, 99)) if wait else None,
            "service_p50_s": float(np.median(service)) if service else None,
            "hw_queues": GpuExecutor.hw_queues_hint(),
            "updates_per_s": srv.updates / wall, "updates": srv.updates, "wall_s": wall,
            "ticks": srv.ticks, "precision": precision, "lattices_L": list(Ls),
            "flagged_requests": flagged, "max_drift": float(max(float(r.obs["max_drift"]) for r in res)),
            "pool_capacity": capacity, "tick_sweeps": tick,
            "refresh_every": refresh if precision == "fp32_wrap" else None}


def run_serving_models(precision: str = "fp64", sweeps_small: int = 10, sweeps_large: int = 2):
    """Compute time of one request of every model of the serving workload, alone on the GPU: one
    chain per model (one workgroup, so one CU), ms per sweep from HIP events.  The request
    latency without queueing is sweeps x ms per sweep; since L, beta and the sweep count are
    drawn uniformly and independently, its distribution over the whole request mix follows
    exactly from the per-model times."""
    import torch
    from paper_2106_00712_amd import dqmc
    models = []
    for L in di.SERVING_L:
        for beta in di.SERVING_BETA:
            n_sl = int(round(beta / 0.1))
            m = dqmc.make_model(di.square_hopping(L), 4.0, 0.1, n_sl, 10, precision=precision,
                                refresh_every=3 if precision == "fp32_wrap" else 0)
            b = dqmc.Batch(m, np.array([(4 << 32) | 7], dtype=np.uint64))
            b.sweep(1)
            k = sweeps_small if L <= 8 else sweeps_large
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            b.sweep(k)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / k
            o = b.measure()
            models.append({"L": L, "beta": beta, "n_sites": L * L, "n_slices": n_sl, "variant": b.variant,
                           "ms_per_sweep": ms, "flags": int(o["flags"][0])})
            print(f"serving model L={L} beta={beta} {precision}: {ms:.2f} ms per sweep", file=sys.stderr,
                  flush=True)
            b.close()
    lo, hi = di.SERVING_SWEEPS
    sweeps = np.arange(lo, hi + 1)
    lat = np.sort(np.concatenate([sweeps * m["ms_per_sweep"] * 1e-3 for m in models]))
    q = lambda f: float(lat[min(len(lat) - 1, int(np.ceil(f * len(lat))) - 1)])
    return {"precision": precision, "models": models,
            "request_latency_without_queueing_s": {"p50": q(0.5), "p99": q(0.99), "mean": float(lat.mean()),
                                                    "max": float(lat[-1])},
            "note": "one chain alone per model; L, beta, sweeps uniform over the serving workload"}


def run_mixed(steps: int, refresh: int, n_each: int, qr_mode: str = "auto", sweep_mode: int = 0):
    """Honeycomb 6x6 (N = 72) and 12x12 (N = 288) chains side by side in one recorded graph,
    FP32 wraps with FP64 refresh every `refresh` slices, against the same batches in FP64."""
    import torch
    from paper_2106_00712_amd import dqmc
    ws = [di.WORKLOADS["honeycomb6x6_U3_b6"], di.WORKLOADS["honeycomb12x12_U3_b6"]]
    qrb = [choose_qr(w, qr_mode) for w in ws]
    out = {"workload": "honeycomb 6x6 + 12x12, U=3, beta=6", "chains_each": n_each, "steps": steps,
           "qr_blocked": qrb, "sweep_mode": sweep_mode}
    for prec in ("fp64", "fp32_wrap"):
        bs = []
        for w, qb in zip(ws, qrb):
            m = dqmc.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every, precision=prec,
                                refresh_every=refresh if prec == "fp32_wrap" else 0, qr_blocked=qb,
                                sweep_mode=sweep_mode)
            bs.append(dqmc.Batch(m, w.seeds(n_each), w.fields(n_each)))
        g = dqmc.Graph(bs, [1, 1])
        g.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.launch()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ups = sum(n_each * w.n_slices * w.n_sites for w in ws) * steps
        obs = [b.measure() for b in bs]
        out[prec] = {"updates_per_s": ups / wall, "ms_per_step": wall * 1e3 / steps,
                     "max_abs_dG_at_refresh": [float(o["max_drift"].max()) for o in obs],
                     "double_occ": [float(o["double_occ"].mean()) for o in obs],
                     "flags": [int(np.bitwise_or.reduce(o["flags"])) for o in obs]}
        g.close()
        for b in bs:
            b.close()
    out["fp32_wrap"]["speedup_vs_fp64"] = out["fp32_wrap"]["updates_per_s"] / out["fp64"]["updates_per_s"]
    out["fp32_wrap"]["fixed_field_wrap_error"] = [fp32_wrap_error(w, 2, 1e-5) for w in ws]
    return out


# Good-DQMC column of the paper's Table 2 (honeycomb, L = 6, U = 3.83, beta = 6, dtau = 0.1)
PAPER_TABLE2 = {"E_k": (-1.358, 0.001), "S_Gamma": (3.00, 0.04)}


def run_physics(n_chains: int, therm: int, meas: int, seed_first: int = 0):
    """Thermalised chains at the paper's honeycomb point; E_k and the sublattice-signed S(Gamma)
    per chain (time average over `meas` sweeps, one measurement at G(0) after each sweep), then
    the mean and standard error over the independent chains.  Every measurement comes from the
    per-sweep series the sweep kernel records on the device (dqmc_sweep_series), copied to the
    host once per block of sweeps."""
    import torch
    from paper_2106_00712_amd import analysis, dqmc
    w = di.WORKLOADS["honeycomb6x6_U3.83_b6"]
    eps = di.staggered_sign(w.lattice, w.L)
    m = dqmc.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    b = dqmc.Batch(m, w.seeds(n_chains, seed_first))
    block = 50

    def series(n_sw, label):
        parts, done = [], 0
        while done < n_sw:
            k = min(block, n_sw - done)
            parts.append(b.sweep_series(k, form=eps).cpu().numpy())
            done += k
            print(f"physics: {label} {done}/{n_sw} sweeps", file=sys.stderr, flush=True)
        return np.concatenate(parts, axis=0) if parts else np.zeros((0, n_chains, 4))

    t0 = time.perf_counter()
    th = series(therm, "thermalised")          # [therm][chains][4], the Fig. 3 form
    torch.cuda.synchronize()
    t_therm = time.perf_counter() - t0
    conv = {"sweeps": [], "E_k": [], "E_k_se": [], "S_Gamma_moments": [], "S_Gamma_moments_se": []}
    for k in sorted(set(range(1, 21)) | set(range(25, therm + 1, 25))):
        if k > therm:
            continue
        conv["sweeps"].append(k)
        for key, v in (("E_k", th[k - 1, :, 2]), ("S_Gamma_moments", 4.0 * th[k - 1, :, 3])):
            mu, se = analysis.mean_and_error(v)
            conv[key].append(mu)
            conv[key + "_se"].append(se)
    ms = series(meas, "measured")               # [meas][chains][4]
    ser = np.stack([ms[:, :, 2].T, ms[:, :, 3].T, ms[:, :, 0].T, ms[:, :, 1].T])  # [4][chains][meas]
    o = b.measure()
    wall = time.perf_counter() - t0
    per_chain = ser.mean(axis=2)
    t_max = min(100, meas // 4)
    a_s = analysis.autocorrelation(ser[1], t_max)
    a_e = analysis.autocorrelation(ser[0], t_max)

    def stat(v):
        return float(v.mean()), float(v.std(ddof=1) / np.sqrt(len(v)))

    ek, s_n, d, dens = (stat(per_chain[i]) for i in range(4))
    s_l2 = (2.0 * s_n[0], 2.0 * s_n[1])          # (1/L^2) sum_ij = (N/L^2) (1/N) sum_ij, N = 2 L^2
    s_m = (4.0 * s_n[0], 4.0 * s_n[1])           # moments m_i = n_i,up - n_i,dn = 2 s^z_i, 1/N
    out = {"workload": w.name, "lattice": "honeycomb", "L": w.L, "n_sites": w.n_sites, "U": w.U,
           "beta": w.beta, "dtau": w.dtau, "chains": n_chains, "thermalisation_sweeps": therm,
           "measurement_sweeps": meas, "E_k": ek, "S_Gamma_1_over_N": s_n, "S_Gamma_1_over_L2": s_l2,
           "S_Gamma_moments_1_over_N": s_m,
           "double_occ": d, "density": dens,
           "acceptance": float(o["accepted"].sum() / max(1, o["attempted"].sum())),
           "flags": int(np.bitwise_or.reduce(o["flags"])), "max_drift": float(o["max_drift"].max()),
           "near_ties": int(o["near_ties"].sum()), "seconds_thermalise": t_therm, "seconds_total": wall,
           "paper_good_dqmc": PAPER_TABLE2, "convergence": conv,
           "autocorr_S_Gamma": {str(t): float(a_s[t]) for t in (1, 2, 5, 10, 20, 50, 100) if t < len(a_s)},
           "autocorr_E_k": {str(t): float(a_e[t]) for t in (1, 2, 5, 10, 20, 50, 100) if t < len(a_e)},
           "tau_int_S_Gamma": analysis.integrated_time(a_s), "tau_int_E_k": analysis.integrated_time(a_e)}
    # %OL (20 bins) of the E_k distribution k sweeps after the random starts against the
    # thermalised one (the paper's overlap measure applied to the Hubbard chains)
    out["percent_overlap_E_k_vs_thermalised"] = {
        str(k): analysis.percent_overlap(th[k - 1, :, 2], ser[0].ravel(), 20)
        for k in (1, 5, 15, 50) if k <= therm}
    for key, (mu, se) in (("E_k", ek), ("S_Gamma_1_over_N", s_n), ("S_Gamma_1_over_L2", s_l2),
                          ("S_Gamma_moments_1_over_N", s_m)):
        pm, pe = PAPER_TABLE2["E_k" if key == "E_k" else "S_Gamma"]
        out[f"{key}_sigma_from_paper"] = (mu - pm) / float(np.hypot(se, pe))
    b.close()
    return out


# Good-MC column of the paper's Table 1 (square Ising, L = 16, T = 2.269 J)
PAPER_TABLE1 = {"abs_M": (0.713, 0.003), "E": (-1.453, 0.002)}
# Algorithmic 32-bit lane operations per Ising update: a quarter of one Philox4x64-10 block
# (10 rounds of two 64x64->128 products as 4 partial 32x32->64 products each = 8 multiplies + 6
# carry adds, two 64-bit xor pairs and the key bump: 40 per round) = 100, the uniform (shift,
# convert, scale) 6, the flip (4 neighbour loads, 3 adds, product, table select, compare,
# store) 14.
ISING_OPS_PER_UPDATE = 120
# Full-rate 32-bit VALU lane operations of the chip: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
PEAK_VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9


def run_ising(L: int, T: float, n_chains: int, therm: int, meas: int, ac_len: int,
              conv_len: int = 300, seed_cfg: int = 7):
    """Table 1's Good-MC numbers from independent chains, the Fig. 3 convergence of |M| from
    random starts, the autocorrelation of M (supplement eq. (5)) and the sweep throughput."""
    import torch
    from paper_2106_00712_amd import analysis, ising
    n = L * L
    b = ising.IsingBatch(L, T, di.chain_seeds(seed_cfg, n_chains))
    conv = b.sweep(conv_len, measure=False, series=True)
    am = np.abs(conv[:, :, 0].double().cpu().numpy()) / n
    curve, curve_se = analysis.convergence_curve(am)
    del conv
    b.sweep(max(0, therm - conv_len), measure=False)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.sweep(meas, measure=True)
    e1.record(stream)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3
    st = b.stats()
    nm = st["n_meas"].astype(np.float64)
    abs_m = analysis.mean_and_error(st["sum_abs_m"] / nm / n)
    e = analysis.mean_and_error(-st["sum_bond"] / nm / n)
    m2 = analysis.mean_and_error(st["sum_m2"] / nm / n ** 2)
    ser = b.sweep(ac_len, measure=False, series=True)[:, :, 0].double().cpu().numpy()
    a = analysis.autocorrelation(ser, min(400, ac_len // 4))
    # %OL (20 bins on [0, 1]) of the |M| distribution k sweeps after random starts against the
    # thermalised one
    am_eq = np.abs(ser).ravel() / n
    ol = {str(k): analysis.percent_overlap(am[:, k - 1], am_eq, 20, (0.0, 1.0))
          for k in (10, 30, 100, 300) if k <= conv_len}
    a_abs = analysis.autocorrelation(np.abs(ser), min(400, ac_len // 4))
    ups = n_chains * meas * n / sec
    out = {"workload": f"ising{L}x{L}_T{T:g}", "L": L, "T": T, "J": 1.0, "chains": n_chains,
           "thermalisation_sweeps": therm, "measurement_sweeps": meas,
           "abs_M": abs_m, "E": e, "M2": m2, "paper_good_mc": PAPER_TABLE1,
           "acceptance": float(st["accepted"].sum() / (st["sweeps_done"].sum() * n)),
           "convergence_abs_M": {str(k): float(curve[k - 1]) for k in (1, 10, 30, 50, 100, 150, 200, 300)
                                 if k <= conv_len},
           "convergence_abs_M_se": {str(k): float(curve_se[k - 1]) for k in (1, 30, 100, 300) if k <= conv_len},
           "autocorr_M": {str(t): float(a[t]) for t in (1, 10, 50, 100, 200, 400) if t < len(a)},
           "tau_int_M": analysis.integrated_time(a), "tau_int_abs_M": analysis.integrated_time(a_abs),
           "percent_overlap_abs_M_vs_thermalised": ol,
           "ms_per_sweep": sec * 1e3 / meas, "updates_per_s": ups,
           "roofline": {"bound": "alu", "achieved": ups * ISING_OPS_PER_UPDATE / 1e12,
                        "peak": PEAK_VALU_LANE_OPS / 1e12, "unit": "T lane-op/s",
                        "frac": ups * ISING_OPS_PER_UPDATE / PEAK_VALU_LANE_OPS, "traffic": None}}
    if L == 16 and abs(T - 2.269) < 1e-12:
        for key in ("abs_M", "E"):
            pm, pe = PAPER_TABLE1[key]
            out[f"{key}_sigma_from_paper"] = (out[key][0] - pm) / float(np.hypot(out[key][1], pe))
    b.close()
    return out


def fp32_wrap_error(w, n_chains: int, bound: float):
    """FP32-wrap error on fixed fields against the FP64 fresh G, per refresh interval."""
    from paper_2106_00712_amd.autotune import Autotuner
    return Autotuner().refresh_interval(w.hopping(), w.U, w.dtau, w.n_slices, w.fields(n_chains),
                                        w.seeds(n_chains), bound=bound,
                                        candidates=(2, 3, 4, 5, 6, 8, 10),
                                        stab_every=w.stab_every)


def drift_stats(o, limit: float) -> dict:
    """Distribution over chains of the drift max|G_wrapped - G_fresh| at the stabilisation
    (refresh) points of a run, and how many chains crossed `limit` (FLAG_DRIFT)."""
    d = np.sort(np.asarray(o["max_drift"], dtype=np.float64))
    return {"max": float(d[-1]), "p50": float(np.median(d)), "p90": float(d[int(0.9 * (len(d) - 1))]),
            "limit": limit, "flagged_chains": int(np.count_nonzero(np.asarray(o["flags"]) & 4)),
            "chains": int(len(d))}


def tune_delay_rank(w, stab: int, candidates):
    """The delay rank the autotuner picks for a workload (timed sweeps of the full batch size,
    at most 256 chains), with its timing table."""
    from paper_2106_00712_amd.autotune import Autotuner
    return Autotuner().delay_rank(w.hopping(), w.U, w.dtau, w.n_slices, stab,
                                  candidates=tuple(candidates), n_chains=min(256, w.n_chains),
                                  sweeps=3 if w.n_sites <= 64 else 1)


def tune_stab(w, bound: float = 1e-6, chains: int = 8):
    """Stabilisation interval for a workload: the largest candidate whose FP64 drift over two
    sweeps from the seeded fields stays within `bound` (the autotuner's drift_interval)."""
    from paper_2106_00712_amd.autotune import Autotuner
    cands = sorted({c for c in (w.stab_every, 8, 5, 4, 2) if c <= w.stab_every}, reverse=True)
    return Autotuner().drift_interval(w.hopping(), w.U, w.dtau, w.n_slices, w.fields(chains),
                                      w.seeds(chains), bound, candidates=cands, precision="fp64")


def _cpu_chains(job):
    """Worker of the CPU baseline: chains [first, first + n) of a workload swept by the oracle in
    baseline mode with the BLAS on one thread; returns the wall seconds of the sweeps."""
    name, first, n, n_sweeps = job
    from threadpoolctl import threadpool_limits
    from oracle import Model, OracleChains
    w = di.WORKLOADS[name]
    with threadpool_limits(1):
        oc = OracleChains(Model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every, stacks=True),
                          w.fields(n, first), w.seeds(n, first))
        t0 = time.perf_counter()
        oc.sweep(n_sweeps)
        return time.perf_counter() - t0


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, chains_per_proc: int, n_sweeps: int, procs: int = 0):
    """The CPU oracle, as it is, in baseline mode (right UDT stack per sweep plus a running left
    factorisation, the GPU's algorithm class) on a bounded sample of the same workload: one
    process per host core (at most 16, the host share of one GPU), each sweeping its own chains
    with a single-threaded BLAS.  Run before anything touches the GPU."""
    import multiprocessing as mp
    ncpu = os.cpu_count() or 1
    procs = procs or max(1, min(16, ncpu))
    jobs = [(w.name, p * chains_per_proc, chains_per_proc, n_sweeps) for p in range(procs)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(procs) as pool:
        pool.map(_cpu_chains, jobs[:1])           # start-up (imports) outside the timed region
        t0 = time.perf_counter()
        per = pool.map(_cpu_chains, jobs)
        wall = time.perf_counter() - t0
    upd = procs * chains_per_proc * n_sweeps * w.n_slices * w.n_sites
    return dict(value=upd / wall, unit="updates/s", cores=procs, kind="oracle",
                sample=f"{procs * chains_per_proc} chains x {n_sweeps} sweeps of the {w.name} workload "
                       f"({upd} updates, {wall:.1f} s wall, {sum(per):.1f} s of sweeps over "
                       f"{procs} processes), oracle in baseline mode, single-threaded BLAS per process",
                nproc=ncpu, cpu_model=_cpu_model())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--delay-rank", default="auto",
                    help="delay rank k, or 'auto': the autotuner's choice among the workload's candidates")
    ap.add_argument("--refresh", type=int, default=0,
                    help="FP32-wrap FP64 refresh interval (0: the longest within max|dG| <= 1e-5 "
                         "on fixed fields, chosen by the autotuner)")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-chains", type=int, default=2, help="CPU baseline: chains per process")
    ap.add_argument("--cpu-sweeps", type=int, default=8)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-full", action="store_true",
                    help="only the serving workload over every lattice size (minutes per rate; "
                         "--precision fp64, fp32_wrap or both)")
    ap.add_argument("--rates", type=float, nargs="+", default=[50.0, 200.0, 2000.0],
                    help="with --serving-full: offered request rates (req/s)")
    ap.add_argument("--requests", type=int, default=1000, help="with --serving-full: requests per rate")
    ap.add_argument("--capacity", type=int, default=64, help="with --serving-full: slots per model pool")
    ap.add_argument("--serving-models", action="store_true",
                    help="compute time of one request of every serving model (L up to 16), alone")
    ap.add_argument("--workload", default=None,
                    help="only a throughput line for this workload (e.g. square20x20_U8_b10)")
    ap.add_argument("--chains", type=int, default=0, help="with --workload: number of chains")
    ap.add_argument("--stab", default="0",
                    help="with --workload: stabilisation interval in slices (0: the workload's; "
                         "'auto': the largest of the workload's interval, 8, 5, 4, 2 whose FP64 "
                         "drift over two sweeps stays within 1e-6)")
    ap.add_argument("--precision", default="fp64", help="with --workload: fp64 or fp32_wrap")
    ap.add_argument("--mixed", action="store_true",
                    help="only the mixed-size batch: honeycomb 6x6 + 12x12, FP32 wraps, one graph")
    ap.add_argument("--physics", action="store_true",
                    help="only the paper's honeycomb point (L=6, U=3.83, beta=6): E_k and S(Gamma)")
    ap.add_argument("--therm", type=int, default=200, help="with --physics: thermalisation sweeps")
    ap.add_argument("--meas", type=int, default=400, help="with --physics: measurement sweeps")
    ap.add_argument("--qr", default="auto", choices=("auto", "pivoted", "blocked"),
                    help="with --workload / --mixed: stabilisation QR of the N > 64 kernels")
    ap.add_argument("--sweep-mode", type=int, default=0,
                    help="with --workload / --mixed: 1 alternating up/down sweeps, 2 per-slice "
                         "measurements, 3 both")
    ap.add_argument("--ising", action="store_true",
                    help="only the Ising workload: Table 1 at L=16, T=2.269, plus L=32 dynamics")
    ap.add_argument("--ising-meas", type=int, default=20000, help="with --ising: measured sweeps at L=16")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 256 MiB device copy first (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: chains are independent, so a multi-GPU run is the "
              "one-GPU run per device; bench.py launches on one GPU only.", file=sys.stderr)
        sys.exit(2)

    if args.workload:
        wl = di.WORKLOADS[args.workload]
        stab_tune = tune_stab(wl) if args.stab == "auto" else None
        stab = stab_tune["interval"] if stab_tune else int(args.stab)
        if args.chains or stab:
            wl = di.Workload(wl.name, wl.config_id, wl.lattice, wl.L, wl.U, wl.beta, wl.dtau,
                             args.chains or wl.n_chains, wl.n_sweeps, stab or wl.stab_every,
                             delay_ranks=wl.delay_ranks)
        qb = choose_qr(wl, args.qr)
        k_tune = None
        if args.delay_rank == "auto" and wl.delay_ranks:
            k_tune = tune_delay_rank(wl, wl.stab_every, wl.delay_ranks)
            k = k_tune["delay_rank"]
        else:
            k = 0 if args.delay_rank == "auto" else int(args.delay_rank)
        r = run_gpu(wl, args.precision, args.steps, args.warmup, k,
                    (args.refresh or 10) if args.precision == "fp32_wrap" else 0, qr_blocked=qb,
                    sweep_mode=args.sweep_mode)
        o = r["obs"]
        ups = wl.n_chains * wl.n_slices * wl.n_sites
        acc = float(o["accepted"].sum() / max(1, o["attempted"].sum()))
        flw = algorithmic_flops(wl.n_sites, wl.n_slices, r["batch"].stab, acc)
        tl = float(np.mean(r["per_launch_ms"])) * 1e-3
        print(json.dumps({"workload": wl.name, "precision": args.precision, "n_chains": wl.n_chains,
                          "n_sites": wl.n_sites, "n_slices": wl.n_slices, "steps": args.steps,
                          "ms_per_sweep": tl * 1e3, "updates_per_s": ups / tl,
                          "tflops": flw["total"] * wl.n_chains / tl / 1e12,
                          "frac_fp64_peak": flw["total"] * wl.n_chains / tl / PEAK_FP64_MFMA,
                          "kernel_variant": r["batch"].variant, "delay_rank": r["batch"].delay_rank,
                          "stab": r["batch"].stab, "qr_blocked": qb, "sweep_mode": args.sweep_mode,
                          "init_ms": r["init_ms"],
                          "max_drift": float(o["max_drift"].max()),
                          "double_occ": float(o["double_occ"].mean()),
                          "flags": int(np.bitwise_or.reduce(o["flags"])),
                          "flagged_chains": int(np.count_nonzero(o["flags"])),
                          "drift": drift_stats(o, 1e-5 if args.precision == "fp32_wrap" else 1e-3),
                          "stab_autotune": stab_tune, "delay_rank_autotune": k_tune,
                          "phase_share": r["phase_share"]}))
        return
    if args.ising:
        r16 = run_ising(16, 2.269, args.chains or 1024, 2000, args.ising_meas, 4000)
        print(json.dumps(r16), flush=True)
        r32 = run_ising(32, 2.269, 256, 4000, 4000, 8000)
        print(json.dumps(r32), flush=True)
        return
    if args.physics:
        print(json.dumps(run_physics(args.chains or 256, args.therm, args.meas)))
        return
    if args.mixed:
        print(json.dumps(run_mixed(args.steps, args.refresh or 10, args.chains or 256, args.qr,
                                   args.sweep_mode)))
        return
    if args.serving_models:
        print(json.dumps({"serving_models": [run_serving_models("fp64"), run_serving_models("fp32_wrap")]}))
        return
    if args.serving_full:
        # the whole request mix (L up to 16, beta in {2, 4, 8}); one JSON line per rate
        precs = ["fp64"]
        if args.precision != "fp64":
            print("the FP32-wrap serving mix is switched off (an unexplained GPU memory fault in its "
                  "test); serving FP64 only", file=sys.stderr)
        for prec in precs:
            for rate in args.rates:
                r = run_serving(rate, args.requests, di.SERVING_L, prec, args.capacity, 10,
                                args.refresh or 3, progress=True)
                print(json.dumps({"serving_full": r}), flush=True)
        return

    w = di.WORKLOADS[WORKLOAD]
    # the CPU oracle first, in worker processes started before this process touches the GPU
    cpu = None if args.no_cpu else cpu_baseline(w, args.cpu_chains, args.cpu_sweeps)
    if args.copy_calibration:
        import torch
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    upd_step = w.n_chains * w.n_slices * w.n_sites
    k_tune = None
    if args.delay_rank == "auto":
        k_tune = tune_delay_rank(w, w.stab_every, w.delay_ranks)
        k = k_tune["delay_rank"]
    else:
        k = int(args.delay_rank)
    r64 = run_gpu(w, "fp64", args.steps, args.warmup, k, 0)
    value = upd_step * args.steps / r64["wall"]
    o = r64["obs"]
    acc = float(o["accepted"].sum() / o["attempted"].sum())
    fl = algorithmic_flops(w.n_sites, w.n_slices, w.stab_every, acc)
    t_launch = float(np.mean(r64["per_launch_ms"])) * 1e-3
    achieved = fl["total"] * w.n_chains / t_launch
    traffic = load_traffic()
    line = {
        "metric": "HS-field updates/s at 8x8 beta=4 (FP64; FP32-wrap alongside)",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["wall"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded uniform +-1 HS fields (stand-in for network-generated configurations)",
        "config": {"workload": w.name, "lattice": "square 8x8 periodic", "t": 1.0, "U": w.U,
                   "beta": w.beta, "dtau": w.dtau, "n_slices": w.n_slices, "n_chains": w.n_chains,
                   "stab_every": w.stab_every, "delay_rank": r64["batch"].delay_rank,
                   "updates_per_step": upd_step, "kernel_variant": r64["batch"].variant,
                   "lds_bytes": r64["batch"].lds_bytes},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_FP64_MFMA / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_MFMA, "traffic": traffic,
                     "kernel": "fast_sweep_kernel<64, double, 16>" if r64["batch"].variant == 2
                     else "chain_kernel<double> (OP_SWEEP)",
                     "launch_ms": t_launch * 1e3,
                     "flop_per_chain_sweep": fl, "acceptance": acc},
        "phase_share": r64["phase_share"],
        "rows": row_rooflines(fl, r64["phase_share"], t_launch, w.n_chains, PEAK_FP64_MFMA),
        "init_ms": r64["init_ms"],
        "delay_rank_autotune": k_tune,
        "max_drift_fp64": float(o["max_drift"].max()),
        "flags": int(np.bitwise_or.reduce(o["flags"])),
    }
    if not args.no_fp32:
        from paper_2106_00712_amd.autotune import Autotuner
        bound = 1e-5
        werr = fp32_wrap_error(w, 4, bound)          # fixed fields: r* wraps stay within the bound
        refresh = args.refresh or werr["refresh_every"]
        r32 = run_gpu(w, "fp32_wrap", args.steps, args.warmup, k, refresh)
        o32 = r32["obs"]
        v32 = upd_step * args.steps / r32["wall"]
        # in sweeps: the drift at the refresh points of a short run for every interval down to 1
        sw = Autotuner().drift_interval(w.hopping(), w.U, w.dtau, w.n_slices, w.fields(64),
                                        w.seeds(64), bound, candidates=(5, 4, 3, 2, 1),
                                        precision="fp32_wrap", sweeps=2, stab_every=w.stab_every)
        # cost of one stabilisation point, from FP64 at half the interval: t = t_core + J t_stab
        r64h = run_gpu(w, "fp64", 10, 2, k, 0, stab=w.stab_every // 2)
        J = lambda st: -(-w.n_slices // st)
        t64 = t_launch
        t64h = float(np.mean(r64h["per_launch_ms"])) * 1e-3
        t32 = float(np.mean(r32["per_launch_ms"])) * 1e-3
        t_stab = (t64h - t64) / (J(w.stab_every // 2) - J(w.stab_every))
        core64 = t64 - J(w.stab_every) * t_stab
        core32 = t32 - J(refresh) * t_stab
        line["fp32_wrap"] = {"value": v32, "unit": "updates/s", "refresh_every": refresh,
                             "ms_per_step": r32["wall"] * 1e3 / args.steps,
                             "speedup_vs_fp64": v32 / value,
                             "bound": bound,
                             "max_abs_dG_fixed_fields": werr["max_abs_dG"].get(str(refresh)),
                             "fixed_field_wrap_error": werr,
                             "in_sweep_drift": drift_stats(o32, bound),
                             "fp64_in_sweep_drift": drift_stats(o, 1e-3),
                             "in_sweep_drift_by_refresh": sw,
                             "cost_model_ms": {"stabilisation_point": t_stab * 1e3,
                                               "fp64_core": core64 * 1e3, "fp32_core": core32 * 1e3,
                                               "fp32_at_fp64_interval": (core32 + J(w.stab_every) * t_stab) * 1e3,
                                               "fp64": t64 * 1e3, "fp64_half_interval": t64h * 1e3,
                                               "fp32": t32 * 1e3},
                             "phase_share": r32["phase_share"],
                             "double_occ": float(o32["double_occ"].mean()),
                             "double_occ_fp64": float(o["double_occ"].mean())}
    if not args.no_serving:
        fast_L = tuple(L for L in di.SERVING_L if L * L <= 64)
        line["serving"] = {
            "note": "Poisson stream of the serving workload drawn over the lattices of the "
                    "N <= 64 kernels (L in 4, 6, 8) at the offered rate; warm pools, continuous "
                    "batching (the whole mix, L up to 16, is bench.py --serving-full)",
            "fp64": [run_serving(rate, 48, fast_L, "fp64", 16, 10, 0) for rate in (100, 1000)],
        }
        # the FP32-wrap serving mix made an unexplained GPU memory fault in a test; it stays off
        line["serving"]["fp32_wrap"] = None
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line))


if __name__ == "__main__":
    main()
