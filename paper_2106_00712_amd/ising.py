"""Python binding of the batched Ising Metropolis sweep (include/ising.h): argument marshalling
only; every step runs in the HIP kernels of libdqmc.so."""
from __future__ import annotations

import ctypes

import numpy as np

from .dqmc import _check, _ptr, _stream, _torch, lib

ISING_OBS_DTYPE = np.dtype([(k, "i8") for k in ("sweeps_done", "accepted", "n_meas", "sum_abs_m",
                                                "sum_m2", "sum_bond", "sum_bond2", "reserved")])


def workspace_bytes(L: int, n_chains: int) -> int:
    return int(lib().ising_workspace_bytes(int(L), int(n_chains)))


class IsingBatch:
    """Independent Metropolis chains of the periodic L x L Ising model, resident on one GPU."""

    def __init__(self, L: int, T: float, seeds, spins=None, J: float = 1.0, device="cuda:0",
                 stream=None, workspace=None):
        torch = _torch()
        self.torch = torch
        self.device = torch.device(device)
        self.L, self.T, self.J = int(L), float(T), float(J)
        seeds = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
        self.n_chains = int(seeds.shape[0])
        nbytes = workspace_bytes(self.L, self.n_chains)
        if nbytes == 0:
            raise ValueError("L must be even and in [2, 64]")
        if workspace is None:
            workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        self._ws = workspace
        base = workspace.data_ptr()
        ptr = (base + 255) & ~255
        avail = workspace.numel() - (ptr - base)
        sp = ctypes.c_void_p(0)
        keep = None
        if spins is not None:
            keep = torch.as_tensor(np.ascontiguousarray(np.asarray(spins, dtype=np.int8))) \
                if not isinstance(spins, torch.Tensor) else spins
            keep = keep.to(device=self.device, dtype=torch.int8).contiguous()
            if keep.numel() != self.n_chains * self.L * self.L:
                raise ValueError(f"spins must be [{self.n_chains}][{self.L * self.L}]")
            sp = _ptr(keep)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().ising_init(ctypes.byref(h), self.L, self.J, self.T, self.n_chains, sp,
                                    seeds.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                    ctypes.c_void_p(ptr), avail, _stream(stream, self.device)))
        self._h = h

    def sweep(self, n_sweeps: int, measure: bool = True, series: bool = False, stream=None):
        """Run n_sweeps sweeps of every chain (one launch); with series=True return the device
        int32 tensor [n_chains][n_sweeps][2] of (M, B) after each sweep."""
        torch = self.torch
        out = None
        if series:
            out = torch.empty((self.n_chains, int(n_sweeps), 2), dtype=torch.int32, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().ising_sweep(self._h, int(n_sweeps), 1 if measure else 0,
                                     _ptr(out) if out is not None else None,
                                     _stream(stream, self.device)))
        return out

    def stats(self, stream=None) -> np.ndarray:
        torch = self.torch
        buf = torch.empty(self.n_chains * ISING_OBS_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().ising_stats(self._h, _ptr(buf), _stream(stream, self.device)))
        return np.frombuffer(buf.cpu().numpy().tobytes(), dtype=ISING_OBS_DTYPE)

    def spins(self, stream=None):
        torch = self.torch
        out = torch.empty((self.n_chains, self.L * self.L), dtype=torch.int8, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().ising_get_spins(self._h, _ptr(out), _stream(stream, self.device)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().ising_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
