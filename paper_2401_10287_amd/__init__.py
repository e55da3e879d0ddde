"""MI355X-native FermiNet VMC hot path (log|psi|, local energy, Metropolis, VMC gradient)."""
