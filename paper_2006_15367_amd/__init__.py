"""MI355X (gfx950) MLFMA matvec for the Helmholtz potential.

``mlfma``     ctypes binding of the C ABI in include/mlfma.h (libmlfma.so)
``autograd``  torch.autograd.Function wrappers (charges and positions)
``workloads`` seeded synthetic point clouds and charges
``build``     in-tree build of libmlfma.so for gfx950
"""
