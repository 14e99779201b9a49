"""MI355X (gfx950) implementation of the multi-speed lattice Boltzmann BGK
scheme with the kinetic diffuse-reflection wall of Meng & Zhang
(arXiv:1209.5201).  The compute path is the HIP library ``liblbm.so``; this
package is its binding."""
from .lbm import *  # noqa: F401,F403
from .lbm import Channel, LbmError, LIB_PATH  # noqa: F401
