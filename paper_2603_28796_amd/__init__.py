"""MI355X-native relaxed-CNF gradient descent (GaloisSAT GPU stage).

Submodules:
  galsat   ctypes binding of libgalsat.so (Problem, GalsatLoss)
  inputs   seeded synthetic CNF workloads and CSR construction
  build    in-tree hipcc build of libgalsat.so
"""


def __getattr__(name):
    if name in ("Problem", "GalsatLoss", "galsat_loss", "GalsatError", "load_library"):
        from . import galsat
        return getattr(galsat, name)
    raise AttributeError(name)
