"""Locality-aware per-element forward-mode AD of mesh energies on MI355X (gfx950)."""
