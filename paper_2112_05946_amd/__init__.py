"""MI355X-native flux reconstruction stochastic Galerkin (FR-SG) hot path.

The numerical work runs in libfrsg.so (hand-written HIP for gfx950) behind the
C ABI of include/fr_sg.h; ``binding`` marshals arguments to it and ``inputs``
defines the workloads.  Importing the package does not load the library;
constructing a ``Solver`` does, and fails if it is missing.
"""


def __getattr__(name):
    if name in ("Solver", "FrsgError", "load_library"):
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
