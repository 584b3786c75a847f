"""CPU FP64 oracles of the DQMC sweep and of the batched Ising Metropolis sweep
(`oracle.ising_oracle`): TEST INFRASTRUCTURE ONLY.

Plain, slow and written to be checked against the paper by eye.  It may be imported only by
tests/, by __graft_entry__.smoke() and by the cpu_baseline leg of bench.py.  It shares no code
with the HIP path (paper_2106_00712_amd) and neither side imports the other; both read their
seeded inputs from dqmc_inputs, which holds none of the method's arithmetic.
"""
from .dqmc_oracle import (Model, OracleChains, hs_nu, kinetic_propagators, slice_B, slice_Binv,
                          udt, udt_exact_pivot, udt_product, green_two_sided, measure_from_green,
                          spin_structure)
from .philox import philox4x64_10, accept_uniform, to_unit

__all__ = ["Model", "OracleChains", "hs_nu", "kinetic_propagators", "slice_B", "slice_Binv", "udt", "udt_exact_pivot",
           "udt_product", "green_two_sided", "measure_from_green", "spin_structure", "philox4x64_10",
           "accept_uniform", "to_unit"]
