"""MI355X (gfx950) 2D electrostatic particle-in-cell hot path for the trench
geometry of Lin & Nishimura (arXiv:1610.03918): integer area-weighting
deposit, masked multigrid-preconditioned CG Poisson solve, field, leapfrog
push with wall absorption and trench-bottom charge build-up.

The kernels live in ``csrc/`` behind the C ABI of ``include/pic.h``;
``pic.py`` is the ctypes binding."""
from .pic import Pic, PicBatch, PicError, lib, make_config  # noqa: F401
