"""LFDPR hot path for MI355X: HIP kernels behind a C ABI, thin Python binding."""
