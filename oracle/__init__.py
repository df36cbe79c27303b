"""CPU oracle of SIM-M (test infrastructure only; never imported by the library)."""
