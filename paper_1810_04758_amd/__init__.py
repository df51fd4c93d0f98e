"""Grid-indexed exact KNN self-join on AMD Instinct MI355X (gfx950)."""
