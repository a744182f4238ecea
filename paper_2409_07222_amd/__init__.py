"""MI355X (gfx950) implementation of the data-parallel hot path of the dual-step
LABS method (arXiv 2409.07222).  The compute lives in liblabs.so (HIP kernels
behind the C ABI of include/labs.h); ``labs`` is its ctypes binding."""
from . import labs  # noqa: F401
