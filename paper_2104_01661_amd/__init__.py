"""MI355X-native masked-semiring sparse library (LAGraph's hot path).

The product is the C-ABI shared library ``liblagr.so`` (``include/lagr.h``)
built from the hand-written HIP sources in ``csrc/``.  ``lagr`` is its thin
ctypes binding; import it explicitly (it raises if the library is not
built -- there is no fallback path).
"""
import os

PACKAGE_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PACKAGE_DIR, "liblagr.so")

