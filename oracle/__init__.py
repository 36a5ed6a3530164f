"""CPU oracle and DMM simulator -- test infrastructure only (see oracle.py)."""
