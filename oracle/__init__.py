"""CPU oracle (test infrastructure only; see lt_oracle.py)."""
