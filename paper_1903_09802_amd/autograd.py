"""C_ext as a differentiable function of the per-voxel permittivity (torch.autograd.Function).

The forward pass calls ``dda_grad_cext`` when the permittivity needs a gradient (one forward
and one adjoint GMRES solve with the same operator and preconditioner, the system matrix
being complex symmetric), else ``dda_solve``.  The backward pass scales the saved gradient,
so a forward + backward costs two solves.  Gradient convention: for the real output C_ext
the returned complex gradient is dC/dRe(eps) + i dC/dIm(eps), as torch expects for complex
leaves of a real loss.
"""

from __future__ import annotations

import numpy as np
import torch

from .dda import Problem, lattice_factor


class DDAExtinction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps, mask, k, d, direction, polarisation, options=None):
        opts = dict(options or {})
        precond = opts.get("precond", 2)
        with Problem(mask, eps.detach(), k, d, **opts) as prob:
            dvec = np.asarray(direction, dtype=np.float64)
            pvec = np.asarray(polarisation, dtype=np.float64)
            if precond != 0:
                # the preconditioner's diagonal at the wave's own lattice factor
                prob.build_preconditioner(lattice_factor(dvec, pvec)[1])
            if ctx.needs_input_grad[0]:
                g, cext, stats, _ = prob.grad_cext(dvec, pvec)
                ctx.save_for_backward(g)
            else:
                out = prob.solve(dvec, pvec, return_c=False, xsec=True)
                cext = float(out["cext"][0])
                stats = out["stats"]
        ctx.stats = stats
        return torch.tensor(cext, dtype=torch.float64, device=eps.device)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out * g, None, None, None, None, None, None


def extinction(eps, mask, k, d, direction, polarisation, **options):
    return DDAExtinction.apply(eps, mask, k, d, direction, polarisation, options)
