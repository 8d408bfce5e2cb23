"""FP64 CPU oracle (test infrastructure only; see se_oracle.py)."""
