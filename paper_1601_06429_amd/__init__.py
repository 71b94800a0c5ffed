"""MI355X-native Voronoi tessellation hot path (per-particle cells of a periodic set)."""
