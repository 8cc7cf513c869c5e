"""Bitslice custom-precision floating point on AMD MI355X (gfx950)."""
