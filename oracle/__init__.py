"""FP64 CPU oracle of the immersed-boundary compressible NS path (test infrastructure only)."""
