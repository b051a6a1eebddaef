"""MI355X-native UV-decomposition ADMM conic solver (hand-written HIP for gfx950)."""
