"""MI355X-native INSPIRIT scheduling hot path (HIP kernels behind a C ABI)."""
