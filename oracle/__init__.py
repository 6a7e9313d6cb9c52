"""FP64 CPU oracle of the hybrid VPL method (test infrastructure only)."""
