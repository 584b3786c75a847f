"""Continuous batching of DQMC chain requests on one GPU.

A request asks for one chain: a square L x L Hubbard lattice at inverse temperature beta, a
number of sweeps and a seed (its starting field is drawn from the seed, or given).  Requests of
the same model (lattice, beta, precision) share a *pool*: one resident batch of chain slots
whose Green's functions, UDT stacks and fields stay in HBM between launches.  Every *tick* the
server

  1. admits waiting requests into free slots of their model's pool (dqmc_init_slots), creating
     the pool first if the HBM budget (sum over pools of capacity x dqmc_chain_bytes) allows;
  2. launches one persistent kernel (dqmc_sweep_counts) on every idle pool with occupied slots,
     each pool on its own stream so that pools of different lattices run side by side on the
     device, every occupied slot advancing by min(tick_sweeps, remaining sweeps);
  3. polls the running pools; a pool whose launch has finished is measured, its finished
     requests leave and their slots free up, and it becomes idle again.

Pools tick independently: a short request is never held back by a slow pool.  A request that
arrives while others are on the GPU starts at the next tick of its pool, in a free slot or a
slot freed by a finished one.  Each chain's trajectory is a function of its seed and field alone
(counter-based random numbers, one workgroup per chain), so its result does not depend on the
pool, the slot or the other requests.

The scheduler (Server) is host logic; the device work goes through an executor.  GpuExecutor
drives libdqmc; tests of the scheduling alone use a simulated executor.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

ModelKey = Tuple[int, float, str]   # (L, beta, precision)


@dataclass
class Request:
    rid: int
    L: int
    beta: float
    sweeps: int
    seed: int
    arrival: float = 0.0                    # seconds since the start of the run
    fields: Optional[np.ndarray] = None     # int8 [n_slices][L*L], or None: drawn from the seed


@dataclass
class Result:
    rid: int
    obs: np.void                   # one dqmc_obs record
    arrival: float
    admitted: float
    finished: float
    fields: Optional[np.ndarray] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class _Slot:
    req: Request
    remaining: int
    admitted: float


@dataclass
class _Pool:
    key: ModelKey
    capacity: int
    handle: object                       # executor's pool object
    slots: Dict[int, _Slot] = field(default_factory=dict)
    running: Optional[np.ndarray] = None  # sweep counts of the launch in flight

    def free_slots(self) -> List[int]:
        return [i for i in range(self.capacity) if i not in self.slots]


class Server:
    """Continuous-batching scheduler over an executor (see the module docstring)."""

    def __init__(self, executor, hbm_budget: int, tick_sweeps: int = 5, pool_capacity: int = 64,
                 precision: str = "fp64", keep_fields: bool = False):
        if tick_sweeps < 1 or pool_capacity < 1:
            raise ValueError("tick_sweeps and pool_capacity must be >= 1")
        self.ex = executor
        self.budget = int(hbm_budget)
        self.tick_sweeps = int(tick_sweeps)
        self.capacity = int(pool_capacity)
        self.precision = precision
        self.keep_fields = keep_fields
        self.pools: Dict[ModelKey, _Pool] = {}
        self.queue: List[Request] = []
        self.used_bytes = 0
        self.ticks = 0
        self.updates = 0

    def _key(self, r: Request) -> ModelKey:
        return (r.L, float(r.beta), self.precision)

    def warm(self, models: Sequence[Tuple[int, float]]):
        """Create the pools of the given (L, beta) models ahead of traffic (a warm server)."""
        for L, beta in models:
            self._pool_for((int(L), float(beta), self.precision))

    def submit(self, r: Request):
        if r.sweeps < 1:
            raise ValueError("a request needs at least one sweep")
        self.queue.append(r)

    def pending(self) -> int:
        return len(self.queue) + sum(len(p.slots) for p in self.pools.values())

    def _pool_for(self, key: ModelKey) -> Optional[_Pool]:
        p = self.pools.get(key)
        if p is not None:
            return p
        per_chain = self.ex.chain_bytes(key)
        cap = self.capacity
        while cap > 1 and self.used_bytes + cap * per_chain > self.budget:
            cap //= 2
        if self.used_bytes + cap * per_chain > self.budget:
            self._release_idle(need=cap * per_chain)
            if self.used_bytes + cap * per_chain > self.budget:
                return None
        p = _Pool(key, cap, self.ex.create_pool(key, cap))
        self.pools[key] = p
        self.used_bytes += cap * per_chain
        return p

    def _release_idle(self, need: int):
        for key in [k for k, p in self.pools.items() if not p.slots]:
            p = self.pools.pop(key)
            self.used_bytes -= p.capacity * self.ex.chain_bytes(key)
            self.ex.release_pool(p.handle)
            if self.used_bytes + need <= self.budget:
                return

    def close(self):
        """Release every pool (its chains' memory; its stream goes back for reuse); requests
        still in the pools or the queue are dropped.  A server that is done should be closed:
        the next server's pools then reuse the same streams, on the same hardware queues, instead
        of new streams that the runtime may put on queues already in use."""
        for key in list(self.pools):
            p = self.pools.pop(key)
            self.used_bytes -= p.capacity * self.ex.chain_bytes(key)
            p.running = None
            self.ex.release_pool(p.handle)
        self.queue = []

    def _admit(self, now: float):
        waiting: List[Request] = []
        grouped: Dict[ModelKey, List[Tuple[int, Request]]] = {}
        for r in self.queue:
            key = self._key(r)
            pool = self._pool_for(key)
            free = pool.free_slots() if (pool is not None and pool.running is None) else []
            if not free:
                waiting.append(r)
                continue
            pool.slots[free[0]] = _Slot(r, r.sweeps, now)    # reserved: the pool is not idle
            grouped.setdefault(key, []).append((free[0], r))
        for key, items in grouped.items():
            self.ex.init_slots(self.pools[key].handle, [s for s, _ in items], [r for _, r in items])
        self.queue = waiting

    def _launch_idle(self):
        for pool in self.pools.values():
            if pool.running is None and pool.slots:
                counts = np.zeros(pool.capacity, dtype=np.int32)
                for s, sl in pool.slots.items():
                    counts[s] = min(self.tick_sweeps, sl.remaining)
                self.ex.launch_tick(pool.handle, counts)
                pool.running = counts
                self.ticks += 1

    def _retire(self, pool: _Pool, now_fn: Callable[[], float]) -> List[Result]:
        counts, pool.running = pool.running, None
        finished = []
        for s, sl in pool.slots.items():
            sl.remaining -= int(counts[s])
            self.updates += int(counts[s]) * pool.key[0] ** 2 * self.ex.n_slices(pool.key)
            if sl.remaining == 0:
                finished.append(s)
        done: List[Result] = []
        if finished:
            obs, fields = self.ex.measure(pool.handle, finished, self.keep_fields)
            t = now_fn()
            for j, s in enumerate(finished):
                sl = pool.slots.pop(s)
                done.append(Result(sl.req.rid, obs[j], sl.req.arrival, sl.admitted, t,
                                   fields[j] if fields is not None else None))
        return done

    def step(self, now_fn: Callable[[], float], wait_until: Optional[float] = None) -> List[Result]:
        """Admit into idle pools, launch every idle pool with work, then retire the pools whose
        launch has finished (waiting for the first to finish, or until wait_until)."""
        self._admit(now_fn())
        self._launch_idle()
        running = [p for p in self.pools.values() if p.running is not None]
        if not running:
            return []
        ready = [p for p in running if self.ex.done(p.handle)]
        if not ready:
            self.ex.wait_any([p.handle for p in running], wait_until, now_fn)
            ready = [p for p in running if self.ex.done(p.handle)]
        out: List[Result] = []
        for p in ready:
            out.extend(self._retire(p, now_fn))
        return out

    def run(self, requests: Sequence[Request], clock: Optional[Callable[[], float]] = None,
            realtime: bool = True, progress: Optional[Callable[[str], None]] = None,
            progress_every: float = 20.0) -> List[Result]:
        """Serve a stream of requests; request.arrival is its time after the start.  With
        realtime=False every request is released at once (a closed loop).  `progress`, if given,
        receives a status line every `progress_every` seconds of the run's clock."""
        t0 = time.perf_counter()
        now = clock or (lambda: time.perf_counter() - t0)
        arrivals = sorted(requests, key=lambda r: r.arrival)
        i, results = 0, []
        t_report = progress_every
        while i < len(arrivals) or self.pending():
            t = now()
            if progress is not None and t >= t_report:
                progress(f"t = {t:.0f} s: {len(results)} of {len(arrivals)} done, "
                         f"{len(self.queue)} queued, {self.pending() - len(self.queue)} on the GPU")
                t_report = t + progress_every
            while i < len(arrivals) and (not realtime or arrivals[i].arrival <= t):
                self.submit(arrivals[i])
                i += 1
            nxt = arrivals[i].arrival if (realtime and i < len(arrivals)) else None
            if not self.pending():
                dt = nxt - t                      # idle: wait for the next arrival
                if clock is None:
                    time.sleep(max(dt, 0.0))
                else:
                    self.ex.advance(max(dt, 0.0))
                continue
            results.extend(self.step(now, wait_until=nxt))
        return results


def latency_stats(results: Sequence[Result]) -> dict:
    lat = np.array([r.latency for r in results])
    if lat.size == 0:
        return {"p50_s": None, "p99_s": None, "mean_s": None, "n": 0}
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "n": int(lat.size)}


# Streams made by dqmc_stream_create, idle, per device.  A released pool hands its stream back
# here instead of destroying it: torch keeps references to a stream past the pool (a pinned
# buffer used in an asynchronous copy on it records an event on that stream when it is freed),
# so the stream must stay valid for the rest of the process.  The next pool reuses it.
_IDLE_STREAMS: Dict[str, list] = {}


class GpuExecutor:
    """Runs the pools through libdqmc: one Batch per pool, one stream per pool.

    Every device call of a pool goes to that pool's stream, host copies included (a tick's sweep
    counts come from a pinned host buffer, the observables go back on the pool's stream), and
    nothing is enqueued on the null stream.  HIP multiplexes streams onto a few hardware queues
    (GPU_MAX_HW_QUEUES per process, 4 by default): pools whose streams share a queue run one after
    the other, and a blocking call (slot initialisation, measurement) on one of them waits for the
    other's whole tick, holding up the host loop meanwhile.  So every pool gets a stream of its
    own making (dqmc_stream_create), not one of torch's pooled streams, whose queues were handed
    out when torch created them; the pools then run side by side when the process has at least
    as many hardware queues as pools.  Streams are reused, never destroyed (see _IDLE_STREAMS).
    `hw_queues_hint` says how many hardware queues the runtime was asked for."""

    def __init__(self, hopping: Callable[[int], np.ndarray], t=1.0, U=4.0, dtau=0.1, stab_every=10,
                 refresh_every=0, delay_rank=0, device="cuda:0"):
        import torch
        from . import dqmc
        self.torch, self.dq = torch, dqmc
        self.hop = hopping          # L -> hopping matrix of the L x L lattice for t = 1
        self.t, self.U, self.dtau = t, U, dtau
        self.stab, self.refresh, self.delay = stab_every, refresh_every, delay_rank
        self.device = torch.device(device)
        self._models = {}

    @staticmethod
    def hw_queues_hint() -> int:
        """Hardware queues per process that the HIP runtime was configured with (its default 4)."""
        import os
        try:
            return int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
        except ValueError:
            return 4

    def n_slices(self, key: ModelKey) -> int:
        return int(round(key[1] / self.dtau))

    def model(self, key: ModelKey):
        m = self._models.get(key)
        if m is None:
            L, beta, prec = key
            m = self.dq.make_model(self.t * self.hop(L), self.U, self.dtau, self.n_slices(key),
                                   self.stab, refresh_every=self.refresh if prec == "fp32_wrap" else 0,
                                   delay_rank=self.delay, precision=prec)
            self._models[key] = m
        return m

    def chain_bytes(self, key: ModelKey) -> int:
        return self.dq.chain_bytes(self.model(key))

    def create_pool(self, key: ModelKey, capacity: int):
        torch = self.torch
        seeds = np.arange(capacity, dtype=np.uint64) + (np.uint64(0xD0C0) << np.uint64(40))
        b = self.dq.Batch(self.model(key), seeds, device=self.device)
        idle = _IDLE_STREAMS.setdefault(str(self.device), [])
        stream = idle.pop() if idle else self.dq.stream_create(self.device)
        pool = {"batch": b, "stream": stream,
                "counts": torch.zeros(capacity, dtype=torch.int32, device=self.device),
                "counts_host": torch.zeros(capacity, dtype=torch.int32, pin_memory=True),
                "done": torch.cuda.Event()}
        # the batch's set-up ran on the current stream: finish it before the pool's stream is used
        torch.cuda.synchronize(self.device)
        return pool

    def release_pool(self, pool):
        pool["stream"].synchronize()
        pool["batch"].close()
        _IDLE_STREAMS.setdefault(str(self.device), []).append(pool["stream"])

    def init_slots(self, pool, slots, reqs):
        torch = self.torch
        b = pool["batch"]
        seeds = np.array([r.seed for r in reqs], dtype=np.uint64)
        fields = None
        if any(r.fields is not None for r in reqs):
            if not all(r.fields is not None for r in reqs):
                raise ValueError("give fields for every request of a tick, or for none")
            fields = torch.as_tensor(np.stack([np.asarray(r.fields, dtype=np.int8) for r in reqs]))
        with torch.cuda.stream(pool["stream"]):
            b.init_slots(slots, seeds, fields, stream=pool["stream"])

    def launch_tick(self, pool, counts):
        # the pinned buffer's previous copy has finished: the pool's last tick is done
        torch = self.torch
        s = pool["stream"]
        pool["counts_host"].numpy()[:] = counts
        with torch.cuda.stream(s):
            pool["counts"].copy_(pool["counts_host"], non_blocking=True)
            pool["batch"].sweep_counts(pool["counts"], stream=s)
            pool["done"].record(s)

    def done(self, pool) -> bool:
        return bool(pool["done"].query())

    def wait_any(self, pools, until, now_fn):
        while not any(p["done"].query() for p in pools):
            if until is not None and now_fn() >= until:
                return
            time.sleep(2e-4)

    def measure(self, pool, slots, keep_fields):
        torch = self.torch
        b = pool["batch"]
        with torch.cuda.stream(pool["stream"]):
            obs = b.measure(stream=pool["stream"])
            fields = None
            if keep_fields:
                fields = b.fields(stream=pool["stream"]).cpu().numpy()[list(slots)]
        return obs[list(slots)], fields

    def advance(self, dt):
        time.sleep(dt)


def poisson_requests(n: int, rate: float, seed: int, Ls=(4, 6, 8, 10, 12, 16), betas=(2.0, 4.0, 8.0),
                     sweeps=(20, 200), config_id: int = 4) -> List[Request]:
    """n requests with exponential inter-arrival times of mean 1/rate; lattice, beta and sweep
    count uniform over the given choices; request r has seed (config_id << 32) | r."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    out = []
    for r in range(n):
        out.append(Request(rid=r, L=int(rng.choice(Ls)), beta=float(rng.choice(betas)),
                           sweeps=int(rng.integers(sweeps[0], sweeps[1] + 1)),
                           seed=(config_id << 32) | r, arrival=float(t[r])))
    return out
