"""MI355X-native matrix-free finite-element Kohn-Sham H.X (HIP for gfx950)."""
