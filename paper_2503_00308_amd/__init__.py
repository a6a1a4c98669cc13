"""Abstract rendering of Gaussian-splat scenes over camera-pose boxes on MI355X (gfx950)."""
