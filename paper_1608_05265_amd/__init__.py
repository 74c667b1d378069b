"""MI355X-native single-precision GEMM (the BLAS sgemm hot path)."""
