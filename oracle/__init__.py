"""CPU reference ("oracle") for one IPC Newton iteration, in float64.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and the
benchmark's CPU-baseline leg may import or run anything in this directory; the
product path (the HIP library and its binding) never does, and shares no code
with it.

It is written to be obviously correct rather than fast:

* energies are the paper's definitions typed out as scalar functions of the
  stencil's vertex positions (``energy.py``);
* gradients and Hessians are the exact derivatives of those functions, taken
  with PyTorch's automatic differentiation on the CPU in float64 (a library
  primitive), and projected onto the PSD cone with a symmetric eigensolver
  (``local.py``);
* the sparsity pattern is a sort/unique of block keys, assembly is a plain
  scatter-add, and the solver is textbook preconditioned CG on a SciPy sparse
  matrix (``pattern.py``, ``assemble.py``, ``pcg.py``, ``newton.py``).
"""
