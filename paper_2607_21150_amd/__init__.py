"""MI355X-native matrix-free phase-field fracture operator (HIP kernels behind a C-ABI)."""
