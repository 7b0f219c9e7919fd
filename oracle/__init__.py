"""FP64 CPU oracle (test infrastructure only; see pf_oracle.c)."""
