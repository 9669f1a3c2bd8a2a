"""CPU oracle for the MRA hot path -- test infrastructure only (see oracle.py)."""
