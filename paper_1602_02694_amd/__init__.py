"""MI355X-native WLS-ENO finite-volume path (Liu & Jiao, arXiv:1602.02694).

The product is ``libwlseno.so`` (C-ABI in ``include/wlseno.h``), built from
``csrc/`` by ``paper_1602_02694_amd.build``.  ``WLSENO`` is the thin Python
binding; it loads the library on first use and raises if it has not been
built -- there is no CPU fallback.
"""

from .wlseno import WLSENO, WLSENOError
from ._native import LibraryMissing, LIB_PATH, EXPORTS

__all__ = ["WLSENO", "WLSENOError", "LibraryMissing", "LIB_PATH", "EXPORTS"]
