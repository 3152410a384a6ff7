"""Seeded synthetic inputs shared by the tests, the bench and the smoke run.

This package holds data only: lens prescriptions (the two printed tables of
the supplement and seeded lens generators), sensor and query descriptions,
and seeded scene generators (all-in-focus images, depth maps, MLP sample
points).  It contains none of the method's arithmetic: no paraxial optics,
no ray tracing, no dual-pixel split, no binning and no rendering.  Both the
CPU oracle and the HIP path consume these objects; neither is imported here.
"""

from .lens import (Surface, Lens, Sensor, PsfQuery, SPHERE, PLANE, STOP,
                   ASPHERE, IDEAL, air, abbe, cauchy)
from . import lenses, scenes, configs

__all__ = ["Surface", "Lens", "Sensor", "PsfQuery", "SPHERE", "PLANE", "STOP",
           "ASPHERE", "IDEAL", "air", "abbe", "cauchy", "lenses"]
