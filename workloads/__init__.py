"""Seeded synthetic SIM-M workloads shared by the oracle, the tests and the benchmark."""
from .gen import (Pencil, make_workload, make_batch, load_config, random_band_pencil,  # noqa: F401
                  convection_diffusion_pencil, planted_pencil, start_vectors, random_band_matrix)
