"""MI355X-native hot path of CLAIRE-style stationary-velocity registration."""
