"""CPU FP64 checker for the GW hot path (test infrastructure only)."""
