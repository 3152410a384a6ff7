"""Plain data descriptions of a lens prescription, a dual-pixel sensor and a
PSF query.  The field meanings follow the column layout of the supplement's
lens tables (Table S1 / Table S2: radius, thickness to the next surface,
material n_d/V_d of the medium after the surface, clear diameter, conic,
a4..a12) and the DP pixel parameters of Sec. 3.1 and Eq. (S1).

Conventions (shared by every consumer of these objects):
  * lengths in millimetres, wavelengths in micrometres;
  * z = 0 at the vertex of the first surface, light travels toward +z;
  * ``c`` is the curvature 1/R (0 for a plane or the aperture stop);
  * ``t`` is the axial distance from this surface's vertex to the next one;
    the last surface's ``t`` is the distance to the sensor plane (used as is
    unless the lens carries a focus distance);
  * ``medium`` names the medium *after* the surface; ``air`` is n = 1;
  * object depths are measured from the first vertex, toward -z.
"""

from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence, Tuple

SPHERE, PLANE, STOP, ASPHERE, IDEAL = 0, 1, 2, 3, 4
KIND_NAMES = {SPHERE: "sphere", PLANE: "plane", STOP: "stop",
              ASPHERE: "asphere", IDEAL: "ideal"}

# Material descriptors: ("cauchy", A, B) means n(lam) = A + B / lam^2 with lam
# in micrometres; ("abbe", n_d, V_d) is the catalogue form printed in the
# supplement's tables.
MAT_CAUCHY, MAT_ABBE = 0, 1


def cauchy(a: float, b: float = 0.0):
    return (MAT_CAUCHY, float(a), float(b))


def abbe(nd: float, vd: float):
    return (MAT_ABBE, float(nd), float(vd))


def air():
    return (MAT_CAUCHY, 1.0, 0.0)


@dataclass
class Surface:
    kind: int                      # SPHERE | PLANE | STOP | ASPHERE | IDEAL
    c: float                       # curvature 1/mm
    t: float                       # thickness to the next vertex (mm)
    semi_diameter: float           # clear semi-diameter (mm)
    medium: Tuple[int, float, float] = field(default_factory=air)
    conic: float = 0.0
    asph: Tuple[float, float, float, float, float] = (0.0, 0.0, 0.0, 0.0, 0.0)
    focal: float = 0.0             # IDEAL surfaces only: focal length (mm)


@dataclass
class Lens:
    surfaces: List[Surface]
    stop: int                      # index of the aperture stop surface
    # If > 0, the stop semi-diameter is rescaled so that the entrance pupil
    # diameter equals EFL / f_number at the reference wavelength.
    f_number: float = 0.0
    # If > 0, the sensor is placed at the paraxial image of an on-axis point
    # at this depth (mm) for the reference wavelength; otherwise the last
    # surface's thickness is the sensor distance.
    focus_depth: float = 0.0
    ref_wavelength: float = 0.55   # micrometres
    object_medium: Tuple[int, float, float] = field(default_factory=air)
    name: str = ""

    def with_surfaces(self, surfaces):
        return replace(self, surfaces=list(surfaces))


DP_SIGMOID, DP_MICROLENS = 0, 1


@dataclass
class Sensor:
    pitch: float                   # DP pixel size ps (mm)
    dp_mode: int = DP_SIGMOID
    sigmoid_k: float = 20.0        # slope of the angular left/right response
    # Microlens model (Sec. 3.1), in units of the pitch; Eq. (S1) values.
    ml_h: float = 0.78
    ml_f: float = 1.44
    ml_w: float = 0.30
    ml_r: float = 0.50
    width_px: int = 0
    height_px: int = 0


SPLAT_BOX, SPLAT_TENT = 0, 1
NORM_NONE, NORM_SUM, NORM_MAX = 0, 1, 2
PUPIL_CONCENTRIC = 0


@dataclass
class PsfQuery:
    fields: Sequence[Tuple[float, float]]   # image-plane points (h_x, h_y) mm
    depths: Sequence[float]                 # object depths from vertex 1, mm
    wavelengths: Sequence[float]            # micrometres
    rays_x: int = 64
    rays_y: int = 64
    seed: int = 0
    jitter: bool = True
    ks: int = 31
    splat: int = SPLAT_BOX
    normalize: int = NORM_NONE
    out_f64: bool = False
    deterministic: bool = False     # bitwise reproducible PSFs (the kernels' mode)

    @property
    def n_points(self):
        return len(self.fields) * len(self.depths) * len(self.wavelengths)

    @property
    def n_rays(self):
        return self.rays_x * self.rays_y
