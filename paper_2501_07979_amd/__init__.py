"""MI355X-native ZDA zone library (arXiv 2501.07979): cylindrical Yee FDTD of
one n-fold Bloch wedge with CPML, soft source, DFT monitors and the adjoint
gradient, behind the C ABI of include/zda.h."""
from . import zda  # noqa: F401
