"""MI355X (gfx950) matrix-free Neo-Hookean operator and p-multigrid solver.

Submodules:
* ``inputs``   - seeded synthetic meshes, fields and materials (numpy only);
* ``binding``  - ctypes binding of ``libhpmg.so`` (Operator, PMG, ``hpmg_*`` functions);
* ``autograd`` - the residual as a ``torch.autograd.Function`` with the adjoint kernel;
* ``problem``  - helpers that move a box mesh to the device and build level operators;
* ``build``    - compiles the HIP library in-tree.

Importing the package loads nothing heavy; ``binding`` loads the shared library on
first use and raises if it is missing.
"""
__all__ = ["inputs", "binding", "autograd", "problem", "build"]
