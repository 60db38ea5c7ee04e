"""MI355X-native Splotch particle renderer (HIP kernels behind a C ABI)."""
