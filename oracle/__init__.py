"""FP64 reference solver (test infrastructure only; see pfo.c)."""
