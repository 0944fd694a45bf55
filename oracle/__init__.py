"""FP64 CPU oracle for the TCUDB join-aggregate (test infrastructure only)."""
