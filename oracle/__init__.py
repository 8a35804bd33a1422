"""Plain FP64 CPU oracle for the batched Ewald path.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg. The library under paper_2507_02888_amd never
imports it, and the oracle shares no code with the library.

Parity unpinned: none -- every entry point is pinned by tests/test_oracle_pins.py
(Madelung constants, alpha independence, invariances, incremental moves,
shell populations of cubic reciprocal lattices for the Jastrow shell index,
the batch driver against the single-walker driver) and by
tests/test_oracle_pins_u.py for the Jastrow u term (hand-evaluated values,
the Kato cusp, the order-C zero at the cutoff, finite differences, images)
and by tests/test_oracle_pins_blip.py for the blip orbitals (partition of
unity, reproduction of linear functions, plane waves at grid nodes, lattice
periodicity, finite differences) and by tests/test_oracle_pins_layers.py
for layered 2D systems (the z = 0 limit, alpha independence at z != 0, the
charged-sheet limit, symmetries, incremental moves).
"""
from .oracle import (  # noqa: F401
    build, lib_path, count_g, gvectors, rho_at, energy, jastrow_derivs, run, run_batch, particles, Variant,
    blip_eval, spins, heights,
)
