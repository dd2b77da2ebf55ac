"""FP64 CPU oracle for the TACAW hot path (test infrastructure only)."""
