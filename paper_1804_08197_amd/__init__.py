"""MI355X (gfx950) stereo volume ray caster: Python side of ``include/sg.h``.

The ray caster, LOD selection, brick pool and compositing run in the HIP
library ``libsg.so`` (sources in ``csrc/``); this package only marshals
arguments (``sg``) and packs linear volumes into brick cores for upload
(``bricks``). Importing it fails if the library has not been built.
"""
from . import sg  # noqa: F401  (raises ImportError when libsg.so is missing)
from .bricks import pack_bricks, upload_volume  # noqa: F401

__all__ = ["sg", "pack_bricks", "upload_volume"]
