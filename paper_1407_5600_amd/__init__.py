"""MI355X-native multiblob immersed-boundary step (gfx950, HIP).

Hot path of Vazquez-Quesada, Balboa Usabiaga & Delgado-Buscalioni,
arXiv:1407.5600: blob-force spreading with the 3-point kernel onto a
periodic staggered grid, the FFT fluid solve with the solenoidal projection,
interpolation back to the blobs, and the springs holding each 13-blob
icosahedral particle together.  The computation lives in ``libmultiblob.so``
(C ABI, ``include/multiblob.h``); this package holds its ctypes binding and
the seeded input generators.
"""
from .binding import (Grid, MultiblobError, Springs, mb_fluid_solve,  # noqa: F401
                      mb_interpolate, mb_interpolate_grad, mb_spread, mb_spring_adjoint,
                      mb_spring_forces, mb_spring_forces_ext, mb_step, mb_step_adjoint,
                      mb_step_ext, mb_step_forced, spring_adjoint, spring_forces, status_string)
