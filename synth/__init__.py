"""Seeded synthetic inputs shared by the library's tests and by the oracle.

This package generates geometry (closed triangle meshes, point sets on plane
curves) and random vectors.
It holds none of the solver's arithmetic: no basis functions, no Green's
function, no tree.  Both sides of every parity test take their inputs from
here and nothing else.
"""
from .meshes import icosphere, capped_cylinder, box_mesh, spheroid, aircraft_like, body_family
from .vectors import complex_normal, mlp_weights
from .curves import smooth_curve, real_normal

__all__ = ["icosphere", "capped_cylinder", "box_mesh", "spheroid", "aircraft_like",
           "body_family", "complex_normal", "mlp_weights", "smooth_curve", "real_normal"]
