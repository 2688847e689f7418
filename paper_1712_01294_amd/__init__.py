"""MI355X (gfx950) meshless finite-mass hydro pass: HIP library + thin binding."""
from . import workloads  # noqa: F401  (numpy-only input generators)

__all__ = ["workloads"]
