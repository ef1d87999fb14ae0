"""Fan-beam coded-aperture coherent-scatter reconstruction on MI355X (gfx950)."""
