"""MI355X-native PageRank pipeline hot path (Dreher et al., arXiv 1603.01876).

K0 generate -> K1 sort -> K2 filter -> K3 PageRank, as HIP kernels for gfx950
behind the C ABI in include/pp.h.  `native` is the thin Python binding;
`workloads` holds the seeded synthetic workload parameters; `build` compiles
the library.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads", "native", "build"]
