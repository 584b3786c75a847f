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

import dqmc_inputs as di  # noqa: E402

PEAK_FP64_MFMA = 78.6e12     # MI355X dense FP64 matrix, FLOP/s
PEAK_FP32_MFMA = 157.3e12    # MI355X dense FP32 matrix, FLOP/s
WORKLOAD = "square8x8_U4_b4"
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2106_00712_amd", "csrc", f)
                  for f in ("dqmc_device.hpp", "dqmc_fast.hpp", "dqmc_stab.hpp", "dqmc_abi.hip")]
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


def run_gpu(w, precision: str, steps: int, warmup: int, delay_rank: int, refresh: int):
    import torch
    from paper_2106_00712_amd import dqmc

    m = dqmc.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every, delay_rank=delay_rank,
                        precision=precision, refresh_every=refresh)
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


def cpu_baseline(w, n_chains: int, n_sweeps: int):
    """The CPU oracle, as it is, on a bounded sample of the same workload."""
    from oracle import Model, OracleChains

    m = Model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    oc = OracleChains(m, w.fields(n_chains), w.seeds(n_chains))
    c0, t0 = time.process_time(), time.perf_counter()
    oc.sweep(n_sweeps)
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    upd = n_chains * n_sweeps * w.n_slices * w.n_sites
    return dict(value=upd / wall, unit="updates/s", cores=max(1, int(round(cpu / wall))),
                kind="oracle",
                sample=f"{n_chains} chains x {n_sweeps} sweeps of the {w.name} workload "
                       f"({upd} updates, {wall:.1f} s wall)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--delay-rank", type=int, default=0)
    ap.add_argument("--refresh", type=int, default=4, help="FP32-wrap FP64 refresh interval")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-chains", type=int, default=12)
    ap.add_argument("--cpu-sweeps", type=int, default=8)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 256 MiB device copy first (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: chains are independent, so a multi-GPU run is the "
              "one-GPU run per device; this build launches on one GPU only.", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        import torch
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = di.WORKLOADS[WORKLOAD]
    upd_step = w.n_chains * w.n_slices * w.n_sites
    r64 = run_gpu(w, "fp64", args.steps, args.warmup, args.delay_rank, 0)
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
        "max_drift_fp64": float(o["max_drift"].max()),
        "flags": int(np.bitwise_or.reduce(o["flags"])),
    }
    if not args.no_fp32:
        r32 = run_gpu(w, "fp32_wrap", args.steps, args.warmup, args.delay_rank, args.refresh)
        o32 = r32["obs"]
        v32 = upd_step * args.steps / r32["wall"]
        line["fp32_wrap"] = {"value": v32, "unit": "updates/s", "refresh_every": args.refresh,
                             "ms_per_step": r32["wall"] * 1e3 / args.steps,
                             "max_abs_dG_vs_fp64": float(o32["max_drift"].max()),
                             "speedup_vs_fp64": v32 / value,
                             "phase_share": r32["phase_share"],
                             "double_occ": float(o32["double_occ"].mean()),
                             "double_occ_fp64": float(o["double_occ"].mean()),
                             "flags": int(np.bitwise_or.reduce(o32["flags"]))}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_chains, args.cpu_sweeps)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
