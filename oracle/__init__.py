"""CPU oracle of the complex Helmholtz Krylov path (test infrastructure only)."""
