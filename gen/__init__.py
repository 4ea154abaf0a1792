"""Seeded synthetic workloads: RE trees, their syntax, and texts of their languages."""
