"""torch.autograd wrapper of the MLFMA matvec: gradients with respect to
the complex charges (the adjoint MLFMA) and the point positions (two field
evaluations), both computed by the HIP library.

    phi = potential(q, xyz, ops)

``ops`` is an :class:`~paper_2006_15367_amd.mlfma.Operators` handle built on
a tree of exactly these positions; ``xyz`` is passed so that autograd can
route a gradient to it (its values are not read here: after moving points,
call ``ops.tree.update_positions(xyz)``, which keeps the tree topology and
refuses moves that leave a leaf box).

Convention (PyTorch, complex): the incoming gradient g = 2 dL/d conj(phi);
returned grad_q = A^H g, grad_xyz[i] = sum_c Re[conj(g_ic) F_q(r_i)_c +
q_ic F_conj(g)(r_i)_c].
"""
import torch


class MLFMAPotential(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, xyz, ops):
        ctx.ops = ops
        ctx.xyz_meta = (xyz.dtype, xyz.device) if isinstance(xyz, torch.Tensor) else None
        ctx.save_for_backward(q)
        return ops.matvec(q)

    @staticmethod
    def backward(ctx, g):
        (q,) = ctx.saved_tensors
        ops = ctx.ops
        g = g.contiguous()
        grad_q = ops.adjoint(g) if ctx.needs_input_grad[0] else None
        grad_x = None
        if ctx.needs_input_grad[1]:
            grad_x = ops.position_gradient(q.detach(), g)
            if ctx.xyz_meta is not None:
                grad_x = grad_x.to(dtype=ctx.xyz_meta[0], device=ctx.xyz_meta[1])
        return grad_q, grad_x, None


def potential(q, xyz, ops):
    """phi = A(xyz) q through the MLFMA, differentiable in q and xyz."""
    return MLFMAPotential.apply(q, xyz, ops)
