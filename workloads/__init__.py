"""Seeded synthetic SIM-M workloads shared by the oracle, the tests and the benchmark."""
from .gen import Pencil, make_workload, make_batch, load_config, random_band_pencil, convection_diffusion_pencil  # noqa: F401
