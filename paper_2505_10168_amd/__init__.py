"""MI355X-native space-time multigrid (STMG) for 1D transient heat conduction.

Subpackages / modules
---------------------
inputs    : seeded synthetic inputs (design fields, loads, request streams)
binding   : ctypes binding of libstmg (the HIP library, include/stmg.h)
autograd  : torch.autograd.Function returning dTheta/drho through the adjoint solve
serving   : continuous-batching request loop over device-resident hierarchies
design    : the optimisation loop of Section 7 (optimality-criteria updates on the GPU)
build     : hipcc build of libstmg.so

Importing the package loads nothing; ``binding`` loads the HIP library and fails
loudly when it has not been built.
"""
__all__ = ["inputs", "binding", "autograd", "serving", "design", "build"]
