"""MI355X-native Monte Carlo simulation of noisy 1D circuits with MPS trajectories and
locally entanglement-optimal unravelings (arXiv 2508.05745).

The package is deliberately import-light: ``inputs`` (seeded synthetic workloads) does not
touch the GPU, and ``mpsb`` (the ctypes binding of the HIP library) loads the native library
only when first used.
"""
