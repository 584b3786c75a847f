"""CPU-side checks of the C ABI: the library loads, exports every declared symbol, sizes its
workspace without a GPU, and the binding refuses to run without one (no CPU fallback)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import dqmc_inputs as di

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b((?:dqmc|ising)_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2106_00712_amd import dqmc
    if not os.path.exists(dqmc.LIB_PATH):
        from paper_2106_00712_amd import build
        build.build()
    return dqmc.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dqmc_init_chains", "dqmc_sweep", "dqmc_measure", "dqmc_workspace_bytes",
                     "dqmc_chain_bytes", "dqmc_sweep_multi", "dqmc_destroy", "dqmc_last_error",
                     "dqmc_spin_structure", "ising_init", "ising_sweep", "ising_stats"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2106_00712_amd import dqmc
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", dqmc.LIB_PATH], capture_output=True, text=True)
    exported = set(re.findall(r"\bT ((?:dqmc|ising)_\w+)", out.stdout))
    assert set(declared_functions()) <= exported


def test_workspace_sizing_without_gpu(lib):
    from paper_2106_00712_amd import dqmc
    w = di.WORKLOADS["square8x8_U4_b4"]
    m = dqmc.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    per = dqmc.chain_bytes(m)
    assert per > 2 * 64 * 64 * 8          # at least both Green's functions
    a, b = dqmc.workspace_bytes(m, 1), dqmc.workspace_bytes(m, 256)
    assert 255 * per <= b - a <= 255 * per + 256 * (8 + 4) + 2 * 256   # plus seed and slot tables
    big = dqmc.make_model(di.square_hopping(20), 8.0, 0.1, 100, 10)
    assert dqmc.chain_bytes(big) > dqmc.chain_bytes(m)


@pytest.mark.parametrize("field,value", [("n_sites", 0), ("n_slices", 0), ("stab_every", 0),
                                         ("precision", 7), ("dtau", -0.1), ("drift_limit", -1.0)])
def test_invalid_model_sizes_to_zero(lib, field, value):
    from paper_2106_00712_amd import dqmc
    m = dqmc.make_model(di.square_hopping(4), 4.0, 0.1, 20, 10)
    setattr(m, field, value)
    assert dqmc.workspace_bytes(m, 4) == 0
    assert b"must" in lib.dqmc_last_error() or b"unknown" in lib.dqmc_last_error() or b"need" in lib.dqmc_last_error()


def test_no_cpu_fallback(lib):
    import torch
    from paper_2106_00712_amd import dqmc
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    m = dqmc.make_model(di.square_hopping(4), 4.0, 0.1, 20, 10)
    with pytest.raises(RuntimeError):
        dqmc.Batch(m, [1])


def test_ising_workspace_sizing_without_gpu(lib):
    from paper_2106_00712_amd import ising
    a, b = ising.workspace_bytes(16, 1), ising.workspace_bytes(16, 1000)
    assert b - a >= 999 * (256 + 64 + 8) - 3 * 256   # spins, counters, seeds (each table 256-aligned)
    for bad in (0, 3, 66):
        assert ising.workspace_bytes(bad, 4) == 0


def test_ising_no_cpu_fallback(lib):
    import torch
    from paper_2106_00712_amd import ising
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        ising.IsingBatch(16, 2.269, [1])
