"""Seeded synthetic input generators shared by the oracle tests, the GPU tests and the benchmark."""
