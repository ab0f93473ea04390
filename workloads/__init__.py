"""Seeded synthetic input generators shared by the oracle tests and the HIP path."""
