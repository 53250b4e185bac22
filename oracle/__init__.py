"""FP64 CPU oracle of the limited lattice Boltzmann step (test infrastructure only)."""
