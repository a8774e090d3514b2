"""FP64 CPU oracle (test infrastructure only; see xsec_oracle)."""
