"""Continuous-batching scheduler (host logic) against a simulated executor: admission by HBM
budget, slot reuse while other chains run, one result per request with its own sweep count,
and latency bookkeeping.  The device side is covered by the GPU serving test."""
import numpy as np
import pytest

from paper_2106_00712_amd.dqmc import OBS_DTYPE
from paper_2106_00712_amd.serving import Request, Server, latency_stats, poisson_requests


class SimExecutor:
    """Pools as dictionaries; a tick costs (max over pools) of sweeps x L^2 x beta x 1 us."""

    def __init__(self):
        self.clock = 0.0
        self.pools = []
        self.live_bytes = 0
        self.max_live = 0
        self.events = []

    def n_slices(self, key):
        return int(round(key[1] / 0.1))

    def chain_bytes(self, key):
        return key[0] ** 2 * 1000

    def create_pool(self, key, cap):
        p = {"key": key, "cap": cap, "slot": {}}
        self.pools.append(p)
        self.live_bytes += cap * self.chain_bytes(key)
        self.max_live = max(self.max_live, self.live_bytes)
        return p

    def release_pool(self, p):
        self.live_bytes -= p["cap"] * self.chain_bytes(p["key"])

    def init_slots(self, p, slots, reqs):
        for s, r in zip(slots, reqs):
            assert 0 <= s < p["cap"]
            p["slot"][s] = {"rid": r.rid, "seed": r.seed, "done": 0}
            self.events.append(("admit", r.rid, self.clock))

    def launch_tick(self, p, counts):
        assert counts.shape == (p["cap"],) and "busy_until" not in p
        for s, c in enumerate(counts):
            if c:
                p["slot"][s]["done"] += int(c)
        p["busy_until"] = self.clock + counts.max() * p["key"][0] ** 2 * p["key"][1] * 1e-6
        self.events.append(("launch", p["key"], self.clock))

    def done(self, p):
        if "busy_until" in p and self.clock >= p["busy_until"]:
            del p["busy_until"]
            return True
        return False

    def wait_any(self, pools, until, now_fn):
        t = min(p["busy_until"] for p in pools)
        if until is not None:
            t = min(t, until)
        self.clock = max(self.clock, t)

    def measure(self, p, slots, keep_fields):
        out = np.zeros(len(slots), dtype=OBS_DTYPE)
        for j, s in enumerate(slots):
            st = p["slot"][s]
            out[j]["sweeps_done"] = st["done"]
            out[j]["attempted"] = st["seed"]
            out[j]["double_occ"] = (st["seed"] % 997) * 1e-3 + st["done"] * 1e-6
        return out, None

    def advance(self, dt):
        self.clock += dt


def _serve(reqs, **kw):
    ex = SimExecutor()
    srv = Server(ex, **kw)
    res = srv.run(reqs, clock=lambda: ex.clock)
    return ex, srv, res


def test_every_request_finishes_once_with_its_sweeps():
    reqs = poisson_requests(120, rate=500.0, seed=1)
    ex, srv, res = _serve(reqs, hbm_budget=10 ** 9, tick_sweeps=5, pool_capacity=8)
    assert sorted(r.rid for r in res) == list(range(120))
    by = {r.rid: r for r in res}
    for q in reqs:
        assert int(by[q.rid].obs["sweeps_done"]) == q.sweeps
        assert int(by[q.rid].obs["attempted"]) == q.seed
        assert by[q.rid].finished >= by[q.rid].admitted >= q.arrival
    assert srv.updates == sum(q.sweeps * q.L ** 2 * int(round(q.beta / 0.1)) for q in reqs)


def test_budget_is_respected_and_idle_pools_are_released():
    reqs = poisson_requests(60, rate=200.0, seed=2)
    budget = 4 * 16 ** 2 * 1000          # four L = 16 chains
    ex, srv, res = _serve(reqs, hbm_budget=budget, tick_sweeps=10, pool_capacity=4)
    assert len(res) == 60
    assert ex.max_live <= budget
    assert srv.used_bytes <= budget


def test_close_releases_every_pool():
    reqs = poisson_requests(30, rate=500.0, seed=3)
    ex, srv, res = _serve(reqs, hbm_budget=10 ** 9, tick_sweeps=5, pool_capacity=4)
    assert len(res) == 30 and ex.live_bytes > 0
    srv.close()
    assert ex.live_bytes == 0 and srv.used_bytes == 0 and not srv.pools and srv.pending() == 0


def test_request_takes_a_freed_slot_while_others_run():
    # capacity 2: A (long) and B (short) start together; C arrives later and must start in B's
    # slot before A has finished
    reqs = [Request(0, 8, 2.0, 200, 11, 0.0), Request(1, 8, 2.0, 10, 12, 0.0),
            Request(2, 8, 2.0, 10, 13, 1e-4)]
    ex, srv, res = _serve(reqs, hbm_budget=10 ** 9, tick_sweeps=5, pool_capacity=2)
    by = {r.rid: r for r in res}
    assert by[2].admitted >= by[1].finished - 1e-12
    assert by[2].finished < by[0].finished
    admits = [e for e in ex.events if e[0] == "admit"]
    assert [a[1] for a in admits] == [0, 1, 2]


def test_results_do_not_depend_on_the_mix():
    reqs = poisson_requests(40, rate=1000.0, seed=3)
    _, _, mixed = _serve(reqs, hbm_budget=10 ** 9, tick_sweeps=7, pool_capacity=3)
    for q in reqs[:5]:
        alone = Request(q.rid, q.L, q.beta, q.sweeps, q.seed, 0.0)
        _, _, res = _serve([alone], hbm_budget=10 ** 9, tick_sweeps=3, pool_capacity=1)
        m = [r for r in mixed if r.rid == q.rid][0]
        assert res[0].obs.tobytes() == m.obs.tobytes()


def test_pools_tick_independently():
    # a long L = 16 request must not hold back a stream of short L = 4 requests
    reqs = [Request(0, 16, 8.0, 100, 1, 0.0)] + [Request(k, 4, 2.0, 10, 100 + k, 1e-3 * k)
                                                 for k in range(1, 9)]
    ex, srv, res = _serve(reqs, hbm_budget=10 ** 9, tick_sweeps=10, pool_capacity=4)
    by = {r.rid: r for r in res}
    short = max(by[k].finished for k in range(1, 9))
    assert short < by[0].finished
    assert all(by[k].latency < 0.5 * by[0].latency for k in range(1, 9))


def test_latency_stats():
    reqs = poisson_requests(50, rate=100.0, seed=4)
    _, _, res = _serve(reqs, hbm_budget=10 ** 9, tick_sweeps=5, pool_capacity=16)
    st = latency_stats(res)
    lat = sorted(r.latency for r in res)
    assert st["n"] == 50 and st["p50_s"] <= st["p99_s"] <= lat[-1] + 1e-12
    assert latency_stats([])["n"] == 0


def test_bad_requests_are_rejected():
    srv = Server(SimExecutor(), hbm_budget=10 ** 9)
    with pytest.raises(ValueError):
        srv.submit(Request(0, 4, 2.0, 0, 1))
    with pytest.raises(ValueError):
        Server(SimExecutor(), hbm_budget=1, tick_sweeps=0)
