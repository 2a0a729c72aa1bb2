"""CPU FP64 oracle (test infrastructure only; see ipfb_oracle)."""
