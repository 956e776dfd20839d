"""FP64 CPU oracle of the Apar-T PIC cycle (test infrastructure only)."""
