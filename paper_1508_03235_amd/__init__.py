"""MI355X-native per-cycle step of a bufferless deflection-routed 2D-mesh multicore
with a statically homed L2 (Kumar & Sahu, arXiv 1508.03235)."""
