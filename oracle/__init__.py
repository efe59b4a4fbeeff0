"""CPU oracle of the blocked linear method (test infrastructure only; see blm_oracle)."""
