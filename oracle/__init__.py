"""FP64 CPU oracle of the diffuse-radiation sweep (test infrastructure only)."""
