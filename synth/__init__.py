"""Seeded synthetic inputs shared by the oracle tests and the HIP path."""
from .bcc_fe import (make_system, cluster_sizes, krylov_vectors, gradient_direction,  # noqa: F401
                     symmetric_direction)
