"""MI355X-native dual-pixel PSF engine: ray-traced DP PSFs, pixel-wise DP
rendering, their adjoints and a bf16 PSF surrogate, all in HIP for gfx950
behind the C ABI of include/sdirt.h.  `sdirt` is the Python binding."""

from . import _abi  # noqa: F401
