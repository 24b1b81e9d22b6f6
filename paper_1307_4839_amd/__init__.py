"""MI355X-native library for the well-balanced 2D Saint-Venant finite-volume step."""
