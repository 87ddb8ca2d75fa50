"""MI355X-native stream-ordered point-to-point and allreduce enqueue library.

The product is the C-ABI shared library ``libmpixs.so`` (header
``include/mpixs.h``), built in-tree for gfx950 by ``build.py``.  The module
``mpixs`` is a thin ctypes binding with the same function names.
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libmpixs.so")
DRIVER_LIB = os.path.join(HERE, "libmpixs_driver.so")
