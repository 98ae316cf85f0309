"""MI355X (gfx950) time stepper of the porous Saint-Venant model on a hexagonal raster.

The method is the explicit finite-volume scheme of Ion, Marinescu and Cruceanu,
"ASTERIX: Module for modelling the water flow on vegetated hillslopes" (arXiv
2406.14933).  The compute path is the HIP library ``lib/libhexsv.so`` (C-ABI in
``include/hexsv.h``); :mod:`paper_2406_14933_amd.hexsv` is its ctypes binding.
"""

__all__ = ["hexsv", "build"]
