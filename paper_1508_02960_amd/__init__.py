"""MI355X-native D3Q19 lattice Boltzmann hot path (arXiv:1508.02960)."""
