"""FP64 scalar oracle of the Chargax environment step (test infrastructure only)."""
