"""MI355X-native lattice Boltzmann hot path (arXiv 2512.12213)."""
