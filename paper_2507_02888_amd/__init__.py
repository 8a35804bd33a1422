"""Batched periodic Ewald energies and single-electron move deltas on MI355X.

The compute path is a HIP library (libewald.so, C ABI declared in
include/ewald.h); `paper_2507_02888_amd.ewald` is its thin ctypes binding and
`paper_2507_02888_amd.workloads` draws the seeded synthetic inputs.
"""
