"""CPU oracle package -- test infrastructure only (see abd_oracle.h)."""
