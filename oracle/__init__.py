"""CPU FP64 oracle (test infrastructure only; see zf_oracle's header)."""
