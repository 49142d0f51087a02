"""CPU oracle of the MMGaP Ising hot path (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package; the GPU library never does.
"""
