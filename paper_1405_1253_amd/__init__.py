"""MI355X-native D2Q37 thermal lattice Boltzmann hot path (placeholder)."""
