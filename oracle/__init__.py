"""FP64 CPU oracle for the MLFMA Helmholtz matvec.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call, link or execute anything in this
package; only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP path: the only module both
sides use is the seeded input generator, which holds none of the method's
arithmetic.

Contents
--------
- ``dense``   : the plain O(N^2) definition of the potential and its gradient
               (paper Sec. 2, Eq. for the Helmholtz potential), in C (FP64,
               OpenMP) behind ctypes.
- ``sphere``  : quadrature on the sphere and the special functions the
               plane-wave MLFMA needs (Gauss-Legendre rule, normalised
               associated Legendre functions, spherical Hankel functions).
- ``mlfma``   : a plain FP64 MLFMA that takes the paper's five stages in the
               paper's order (Sec. 2 list; Sec. 3.2.1-3.2.5): C2M, M2M
               (interpolate, shift, aggregate), M2L, L2L (shift, anterpolate,
               aggregate), L2O, plus the leaf-level near field.

Conventions (kernel sign/scale, sample grids, truncation rule, tree
definition) are the readings listed in the design notes; each function
states the passage it follows.
"""
