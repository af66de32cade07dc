"""MI355X-native bootstrap multigrid (BMG) eigensolver for the P1 surface-FEM
Laplace-Beltrami pencil A u = lambda M u.

The solver is the HIP library libbmg.so (C ABI in include/bmg.h); this package
is its Python binding.
"""
from .bmg import (BMGError, Hierarchy, Server, finest_vertices, EXPORTED, LIB_PATH, status_string, surface_desc,
                  OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, EBUSY, ECANCELED)

__all__ = ["BMGError", "Hierarchy", "Server", "finest_vertices", "EXPORTED", "LIB_PATH", "status_string", "surface_desc"]
