"""MI355X-native hot path of one IPC Newton iteration (stable Neo-Hookean
tetrahedra + log-barrier contact stencils -> 3x3 BSR Hessian -> block-Jacobi
PCG), after "YASPS: A Symbolic Framework for Extensible, High-Performance IPC
Simulation" (ACM TOG 45(4), 2026).

The compute path lives in the HIP library ``libyasps.so`` (C-ABI in
``include/yasps.h``); :mod:`.yasps` is its thin ctypes binding and
:mod:`.synth` builds seeded synthetic inputs.  Importing this package does not
load the library.
"""
