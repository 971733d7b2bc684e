"""Pseudo-spectral Navier-Stokes + Cahn-Hilliard timestep for AMD MI355X (gfx950)."""
