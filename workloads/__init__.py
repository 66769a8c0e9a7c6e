"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark: geometries, material parameter sets, frequency grids and the
workload recipes.  No equation of the response model is evaluated here."""
