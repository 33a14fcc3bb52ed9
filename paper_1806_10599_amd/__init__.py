"""MI355X-native variational FFT homogenization (arXiv:1806.10599 hot path).

The solver lives in the HIP shared library ``libpaper_1806_10599_amd.so``
(C ABI: ``include/rve.h``); ``binding`` is its ctypes wrapper.  Import the
binding explicitly (``from paper_1806_10599_amd.binding import Rve``); this
package init loads nothing so that the build step can run without a GPU.
"""

LIBNAME = "libpaper_1806_10599_amd.so"
