"""Seeded synthetic inputs shared by the oracle tests, the HIP-path tests and the benchmark."""
