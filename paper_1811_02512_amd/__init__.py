"""MI355X-native Newton-Raphson AC power flow (graph-based decomposition of
arXiv 1811.02512): host symbolic analysis + gfx950 HIP kernels behind a C ABI
(include/pf.h).  Import fails loudly if libpf.so has not been built."""
from . import binding  # noqa: F401  (raises ImportError if libpf.so is missing)

__all__ = ["binding"]
