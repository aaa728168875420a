"""MI355X-native Metropolis-Kawasaki lattice sweeps (HIP kernels behind a C ABI)."""
