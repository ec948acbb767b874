"""MI355X (gfx950) implementation of the MLPG discrete-ordinates transport hot path.

``mlpg`` is the ctypes binding of ``libmlpg.so`` (C ABI in ``include/mlpg.h``);
``problem`` sequences the four stage calls for one problem.
"""
from . import mlpg  # noqa: F401
