"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark."""
