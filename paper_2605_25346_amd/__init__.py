"""MI355X-native batched CROWN-style bound propagation (gfx950 HIP kernels behind a C-ABI)."""
