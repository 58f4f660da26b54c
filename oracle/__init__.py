"""FP64 CPU oracle (test infrastructure; never used by the search product)."""
