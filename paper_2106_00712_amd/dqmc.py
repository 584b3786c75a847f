"""Thin ctypes binding of libdqmc.so (include/dqmc.h).

Argument marshalling only: PyTorch supplies device memory (the workspace, fields and output
buffers are torch tensors on the GPU) and streams; every step of the sweep runs in the HIP
kernels of the library.  There is no CPU fallback: without the built library, or without a GPU,
every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdqmc.so")

FP64 = 0
FP32_WRAP = 1
PRECISIONS = {"fp64": FP64, "fp32_wrap": FP32_WRAP}

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENUMERIC", -5: "EBUSY"}
FLAG_NONFINITE, FLAG_NEGATIVE, FLAG_DRIFT, FLAG_SINGULAR = 1, 2, 4, 8


class DqmcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"dqmc {STATUS.get(status, status)}: {msg}")
        self.status = status


class Model(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int32), ("hopping", ctypes.POINTER(ctypes.c_double)),
                ("U", ctypes.c_double), ("mu", ctypes.c_double), ("dtau", ctypes.c_double),
                ("n_slices", ctypes.c_int32), ("stab_every", ctypes.c_int32),
                ("refresh_every", ctypes.c_int32), ("delay_rank", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("qr_blocked", ctypes.c_int32),
                ("sweep_mode", ctypes.c_int32), ("drift_limit", ctypes.c_double)]


OBS_DTYPE = np.dtype([("double_occ", "f8"), ("density", "f8"), ("kinetic", "f8"),
                      ("logdet_up", "f8"), ("logdet_dn", "f8"), ("max_drift", "f8"),
                      ("max_logdet_err", "f8"), ("attempted", "i8"), ("accepted", "i8"),
                      ("near_ties", "i8"), ("sweeps_done", "i8"), ("flags", "i4"),
                      ("reserved", "i4"), ("slice_double_occ", "f8"), ("slice_kinetic", "f8"),
                      ("slice_meas", "i8")])

_lib = None
_vp, _i32, _u64, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_size_t

_SIGS = {
    "dqmc_chain_bytes": (_sz, [ctypes.POINTER(Model)]),
    "dqmc_workspace_bytes": (_sz, [ctypes.POINTER(Model), _i32]),
    "dqmc_init_chains": (_i32, [ctypes.POINTER(_vp), ctypes.POINTER(Model), _i32, _vp,
                                ctypes.POINTER(_u64), _vp, _sz, _vp]),
    "dqmc_sweep": (_i32, [_vp, _i32, _vp]),
    "dqmc_sweep_series": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "dqmc_sweep_multi": (_i32, [ctypes.POINTER(_vp), ctypes.POINTER(_i32), _i32, _vp]),
    "dqmc_measure": (_i32, [_vp, _vp, _vp, _vp]),
    "dqmc_get_fields": (_i32, [_vp, _vp, _vp]),
    "dqmc_spin_structure": (_i32, [_vp, _vp, _vp, _vp]),
    "dqmc_destroy": (_i32, [_vp]),
    "dqmc_last_error": (ctypes.c_char_p, []),
    "dqmc_stream_create": (_i32, [ctypes.POINTER(_vp)]),
    "dqmc_stream_destroy": (_i32, [_vp]),
    "dqmc_batch_info": (_i32, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                               ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "dqmc_init_slots": (_i32, [_vp, ctypes.POINTER(_i32), _i32, _vp, ctypes.POINTER(_u64), _vp]),
    "dqmc_sweep_counts": (_i32, [_vp, _vp, _vp]),
    "dqmc_graph_create": (_i32, [ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_i32), _i32]),
    "dqmc_graph_launch": (_i32, [_vp, _vp]),
    "dqmc_graph_destroy": (_i32, [_vp]),
    "dqmc_run_static": (_i32, [ctypes.POINTER(Model), _i32, _vp, ctypes.POINTER(_u64), _i32, _vp,
                               _vp, _vp, _vp]),
    "dqmc_debug_green": (_i32, [_vp, _i32, _i32, _vp, _vp]),
    "dqmc_debug_ratios": (_i32, [_vp, _i32, _vp, _vp]),
    "dqmc_debug_propagators": (_i32, [_vp, _vp, _vp]),
    "dqmc_debug_phase_ticks": (_i32, [_vp, _vp, _vp]),
    "dqmc_debug_philox": (_i32, [_u64, _u64, _u64, _u64, _u64, _u64, _i32, _vp, _vp]),
    "dqmc_debug_mfma": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    # include/ising.h
    "ising_workspace_bytes": (_sz, [_i32, _i32]),
    "ising_init": (_i32, [ctypes.POINTER(_vp), _i32, ctypes.c_double, ctypes.c_double, _i32, _vp,
                          ctypes.POINTER(_u64), _vp, _sz, _vp]),
    "ising_sweep": (_i32, [_vp, _i32, _i32, _vp, _vp]),
    "ising_stats": (_i32, [_vp, _vp, _vp]),
    "ising_get_spins": (_i32, [_vp, _vp, _vp]),
    "ising_destroy": (_i32, [_vp]),
}


def lib():
    """Load libdqmc.so (built in-tree by build.build()); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise DqmcError(status, lib().dqmc_last_error().decode())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libdqmc needs a ROCm GPU; torch.cuda.is_available() is False")
    return torch


def _stream(stream, device):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def stream_create(device="cuda:0"):
    """A non-blocking HIP stream of the caller's own (dqmc_stream_create), not one of torch's
    pooled streams, as a torch stream object; give it back with stream_destroy."""
    torch = _torch()
    h = ctypes.c_void_p()
    with torch.cuda.device(device):
        _check(lib().dqmc_stream_create(ctypes.byref(h)))
    return torch.cuda.ExternalStream(h.value, device=device)


def stream_destroy(stream):
    """Wait for the stream's work and destroy a stream made by stream_create.  Only once nothing
    that refers to it is alive: torch events recorded on it, and pinned host tensors used in an
    asynchronous copy on it (torch records an event on that stream when such a tensor is freed)."""
    _check(lib().dqmc_stream_destroy(ctypes.c_void_p(stream.cuda_stream)))


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def make_model(hopping, U, dtau, n_slices, stab_every, mu=0.0, refresh_every=0, delay_rank=0,
               precision="fp64", qr_blocked=False, sweep_mode=0, drift_limit=0.0):
    """Build the C model struct; the returned object keeps the host hopping array alive."""
    T = np.ascontiguousarray(np.asarray(hopping, dtype=np.float64))
    if T.ndim != 2 or T.shape[0] != T.shape[1]:
        raise ValueError("hopping must be N x N")
    m = Model()
    m.n_sites = T.shape[0]
    m.hopping = T.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    m.U, m.mu, m.dtau = float(U), float(mu), float(dtau)
    m.n_slices, m.stab_every = int(n_slices), int(stab_every)
    m.refresh_every, m.delay_rank = int(refresh_every), int(delay_rank)
    m.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    m.qr_blocked = 1 if qr_blocked else 0
    m.sweep_mode = int(sweep_mode)
    m.drift_limit = float(drift_limit)
    m._keep = T
    return m


def chain_bytes(model: Model) -> int:
    return int(lib().dqmc_chain_bytes(ctypes.byref(model)))


def workspace_bytes(model: Model, n_chains: int) -> int:
    return int(lib().dqmc_workspace_bytes(ctypes.byref(model), int(n_chains)))


class Batch:
    """A batch of independent DQMC chains of one model, resident on one GPU."""

    def __init__(self, model: Model, seeds, fields=None, device="cuda:0", stream=None,
                 workspace=None):
        torch = _torch()
        self.torch = torch
        self.device = torch.device(device)
        self.model = model
        self.n = model.n_sites
        self.L = model.n_slices
        seeds = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
        self.n_chains = int(seeds.shape[0])
        self.seeds = seeds
        nbytes = workspace_bytes(model, self.n_chains)
        if nbytes == 0:
            _check(-1)
        if workspace is None:
            workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        self._ws = workspace
        base = workspace.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        self._ws_bytes = workspace.numel() - (self._ws_ptr - base)
        if fields is not None:
            if isinstance(fields, torch.Tensor):
                f = fields
            else:
                f = torch.as_tensor(np.ascontiguousarray(np.asarray(fields, dtype=np.int8)))
            f = f.to(device=self.device, dtype=torch.int8).contiguous()
            if tuple(f.shape) != (self.n_chains, self.L, self.n):
                raise ValueError(f"fields must be [{self.n_chains}][{self.L}][{self.n}]")
            self._fields_in = f
            fptr = _ptr(f)
        else:
            self._fields_in = None
            fptr = ctypes.c_void_p(0)
        h = ctypes.c_void_p()
        s = _stream(stream, self.device)
        with torch.cuda.device(self.device):
            _check(lib().dqmc_init_chains(ctypes.byref(h), ctypes.byref(model), self.n_chains, fptr,
                                          seeds.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                          ctypes.c_void_p(self._ws_ptr), self._ws_bytes, s))
        self._h = h
        self._fields_in = None
        k, st, ldsb, var = _i32(), _i32(), _i32(), _i32()
        _check(lib().dqmc_batch_info(h, ctypes.byref(k), ctypes.byref(st), ctypes.byref(ldsb),
                                     ctypes.byref(var)))
        self.delay_rank, self.stab, self.lds_bytes, self.variant = k.value, st.value, ldsb.value, var.value

    @property
    def handle(self):
        return self._h

    def sweep(self, n_sweeps: int, stream=None):
        with self.torch.cuda.device(self.device):
            _check(lib().dqmc_sweep(self._h, int(n_sweeps), _stream(stream, self.device)))

    SERIES = ("double_occ", "density", "kinetic", "structure")

    def sweep_series(self, n_sweeps: int, form=None, stream=None):
        """n_sweeps sweeps, recording every chain's estimators after each sweep on the device:
        a float64 tensor [n_sweeps][n_chains][4] (double occupancy, density, kinetic energy, the
        structure factor of the real form factor `form`, or 0 without one)."""
        torch = self.torch
        out = torch.empty((int(n_sweeps), self.n_chains, 4), dtype=torch.float64, device=self.device)
        f = None
        if form is not None:
            f = torch.as_tensor(np.asarray(form, dtype=np.float64)).to(self.device)
            if f.numel() != self.n:
                raise ValueError(f"form factor has {f.numel()} entries, the lattice {self.n} sites")
            self._form_keep = f
        with torch.cuda.device(self.device):
            _check(lib().dqmc_sweep_series(self._h, int(n_sweeps), _ptr(f) if f is not None else None,
                                           _ptr(out), _stream(stream, self.device)))
        return out

    def init_slots(self, slots, seeds, fields=None, stream=None):
        """Re-initialise the listed chains with new seeds (and fields, else drawn from the seeds)."""
        torch = self.torch
        slots = np.ascontiguousarray(np.asarray(slots, dtype=np.int32))
        seeds = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
        if slots.shape != seeds.shape or slots.ndim != 1:
            raise ValueError("slots and seeds must be 1-D and of equal length")
        fptr, keep = ctypes.c_void_p(0), None
        if fields is not None:
            f = fields if isinstance(fields, torch.Tensor) else torch.as_tensor(
                np.ascontiguousarray(np.asarray(fields, dtype=np.int8)))
            keep = f.to(device=self.device, dtype=torch.int8).contiguous()
            if tuple(keep.shape) != (len(slots), self.L, self.n):
                raise ValueError(f"fields must be [{len(slots)}][{self.L}][{self.n}]")
            fptr = _ptr(keep)
        with torch.cuda.device(self.device):
            _check(lib().dqmc_init_slots(self._h, slots.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                         len(slots), fptr,
                                         seeds.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                         _stream(stream, self.device)))
        del keep

    def sweep_counts(self, counts, stream=None):
        """One launch in which chain c runs counts[c] sweeps (a device int32 tensor [n_chains])."""
        torch = self.torch
        if not isinstance(counts, torch.Tensor) or counts.dtype != torch.int32 or \
                counts.device != self.device or tuple(counts.shape) != (self.n_chains,):
            raise ValueError(f"counts must be an int32 tensor [{self.n_chains}] on {self.device}")
        counts = counts.contiguous()
        self._counts_keep = counts   # alive until the next launch of this batch is enqueued
        with torch.cuda.device(self.device):
            _check(lib().dqmc_sweep_counts(self._h, _ptr(counts), _stream(stream, self.device)))

    def measure(self, green: bool = False, stream=None):
        """Per-chain observables (numpy structured array) and optionally G(0) [c][2][N][N]."""
        torch = self.torch
        obs = torch.empty(self.n_chains * OBS_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
        g = torch.empty((self.n_chains, 2, self.n, self.n), dtype=torch.float64,
                        device=self.device) if green else None
        with torch.cuda.device(self.device):
            st = lib().dqmc_measure(self._h, _ptr(obs), _ptr(g) if g is not None else None,
                                    _stream(stream, self.device))
        if st not in (0, -4):
            _check(st)
        o = np.frombuffer(obs.cpu().numpy().tobytes(), dtype=OBS_DTYPE)
        return (o, g) if green else o

    def spin_structure(self, form, stream=None):
        """(1/N) sum_ij f_i f_j <s^z_i s^z_j> of every chain at G(0) for a real form factor f
        (length N); a device float64 tensor [n_chains], computed asynchronously on the stream."""
        torch = self.torch
        f = torch.as_tensor(np.asarray(form, dtype=np.float64)).to(self.device)
        if f.numel() != self.n:
            raise ValueError(f"form factor has {f.numel()} entries, the lattice {self.n} sites")
        out = torch.empty(self.n_chains, dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().dqmc_spin_structure(self._h, _ptr(f), _ptr(out), _stream(stream, self.device)))
        self._form_keep = f
        return out

    def fields(self, stream=None):
        torch = self.torch
        out = torch.empty((self.n_chains, self.L, self.n), dtype=torch.int8, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().dqmc_get_fields(self._h, _ptr(out), _stream(stream, self.device)))
        return out

    def debug_green(self, slice_: int, n_wraps: int = 0, stream=None):
        torch = self.torch
        out = torch.empty((self.n_chains, 2, self.n, self.n), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().dqmc_debug_green(self._h, int(slice_), int(n_wraps), _ptr(out),
                                          _stream(stream, self.device)))
        return out

    def debug_ratios(self, slice_: int, stream=None):
        torch = self.torch
        out = torch.empty((self.n_chains, 2, self.n), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().dqmc_debug_ratios(self._h, int(slice_), _ptr(out), _stream(stream, self.device)))
        return out

    def propagators(self, stream=None):
        torch = self.torch
        out = torch.empty((2, self.n, self.n), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().dqmc_debug_propagators(self._h, _ptr(out), _stream(stream, self.device)))
        return out

    PHASES = ("right_stack", "wrap", "decide", "panel", "flush", "left_udt", "fresh_g", "sweep",
              "chunk_gemm", "qr", "q_form", "t_gemm", "fresh_gemm", "gauss_jordan", "g_out", "park")

    def phase_seconds(self, stream=None):
        """Per-chain seconds spent in each phase of the sweeps so far ([n_chains][16])."""
        torch = self.torch
        out = torch.zeros((self.n_chains, 16), dtype=torch.int64, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().dqmc_debug_phase_ticks(self._h, _ptr(out), _stream(stream, self.device)))
        return out.cpu().numpy() / 1.0e8

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dqmc_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


STATIC_BYTES = 64 << 20


def run_static(model: Model, seeds, fields=None, n_sweeps: int = 1, green: bool = False,
               get_fields: bool = True, device="cuda:0", stream=None):
    """dqmc_run_static: init, n_sweeps sweeps and the measurement in one call, in the library's
    static device array (no workspace).  Returns (obs, green or None, fields or None); the output
    buffers are allocated here, by the caller of the entry point."""
    torch = _torch()
    dev = torch.device(device)
    seeds = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
    n = int(seeds.shape[0])
    N, L = model.n_sites, model.n_slices
    keep = None
    fptr = ctypes.c_void_p(0)
    if fields is not None:
        f = fields if isinstance(fields, torch.Tensor) else torch.as_tensor(
            np.ascontiguousarray(np.asarray(fields, dtype=np.int8)))
        keep = f.to(device=dev, dtype=torch.int8).contiguous()
        if tuple(keep.shape) != (n, L, N):
            raise ValueError(f"fields must be [{n}][{L}][{N}]")
        fptr = _ptr(keep)
    obs = torch.empty(max(1, n) * OBS_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    g = torch.empty((n, 2, N, N), dtype=torch.float64, device=dev) if green else None
    fo = torch.empty((n, L, N), dtype=torch.int8, device=dev) if get_fields else None
    with torch.cuda.device(dev):
        st = lib().dqmc_run_static(ctypes.byref(model), n, fptr,
                                   seeds.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), int(n_sweeps),
                                   _ptr(obs), _ptr(g) if g is not None else None,
                                   _ptr(fo) if fo is not None else None, _stream(stream, dev))
    if st not in (0, -4):
        _check(st)
    del keep
    o = np.frombuffer(obs.cpu().numpy().tobytes(), dtype=OBS_DTYPE)[:n]
    return o, g, fo


def sweep_multi(batches, n_sweeps, stream=None):
    """Sweep several batches together (one launch each, overlapping on forked streams)."""
    if not batches:
        return
    torch = batches[0].torch
    hs = (ctypes.c_void_p * len(batches))(*[b.handle.value for b in batches])
    ns = (ctypes.c_int32 * len(batches))(*[int(x) for x in n_sweeps])
    dev = batches[0].device
    with torch.cuda.device(dev):
        _check(lib().dqmc_sweep_multi(hs, ns, len(batches), _stream(stream, dev)))


class Graph:
    """A recorded sweep of several batches (one HIP graph); each launch() advances them."""

    def __init__(self, batches, n_sweeps):
        if not batches:
            raise ValueError("need at least one batch")
        self.batches = list(batches)
        self.torch = batches[0].torch
        self.device = batches[0].device
        hs = (ctypes.c_void_p * len(batches))(*[b.handle.value for b in batches])
        ns = (ctypes.c_int32 * len(batches))(*[int(x) for x in n_sweeps])
        g = ctypes.c_void_p()
        with self.torch.cuda.device(self.device):
            _check(lib().dqmc_graph_create(ctypes.byref(g), hs, ns, len(batches)))
        self._g = g

    def launch(self, stream=None):
        with self.torch.cuda.device(self.device):
            _check(lib().dqmc_graph_launch(self._g, _stream(stream, self.device)))

    def close(self):
        if getattr(self, "_g", None) is not None and self._g.value:
            lib().dqmc_graph_destroy(self._g)
            self._g = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def debug_philox(key, ctr, n_blocks, device="cuda:0"):
    torch = _torch()
    out = torch.empty((n_blocks, 4), dtype=torch.uint64, device=device)
    with torch.cuda.device(device):
        _check(lib().dqmc_debug_philox(key[0], key[1], ctr[0], ctr[1], ctr[2], ctr[3], n_blocks,
                                       _ptr(out), _stream(None, torch.device(device))))
    return out


def debug_mfma(a64, b64, a32, b32, device="cuda:0"):
    torch = _torch()
    dev = torch.device(device)
    ta64 = torch.as_tensor(a64, dtype=torch.float64, device=dev).contiguous()
    tb64 = torch.as_tensor(b64, dtype=torch.float64, device=dev).contiguous()
    ta32 = torch.as_tensor(a32, dtype=torch.float32, device=dev).contiguous()
    tb32 = torch.as_tensor(b32, dtype=torch.float32, device=dev).contiguous()
    o64 = torch.zeros((16, 16), dtype=torch.float64, device=dev)
    o32 = torch.zeros((16, 16), dtype=torch.float32, device=dev)
    with torch.cuda.device(dev):
        _check(lib().dqmc_debug_mfma(_ptr(ta64), _ptr(tb64), _ptr(o64), _ptr(ta32), _ptr(tb32),
                                     _ptr(o32), _stream(None, dev)))
    return o64, o32
