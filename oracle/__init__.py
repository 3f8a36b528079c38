"""FP64 CPU oracle (test infrastructure only; see henn_oracle.py)."""
