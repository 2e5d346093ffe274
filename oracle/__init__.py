"""FP64 CPU oracle (test infrastructure only; see chi0_oracle)."""
