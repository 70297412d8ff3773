"""torch.autograd.Function around the library's free-energy gradient.

FermiFreeEnergy.apply(values, engine, T, mu, n_terms) returns the probe estimate
F~ of tr g(H) for H with the engine's block pattern and the given block values;
its backward multiplies the incoming gradient by dF~/dH, which the library's
reverse-Clenshaw kernels produce in the forward call (paper: Analytical
free-energy derivatives).  Composing it with a torch-built H(R) gives
Hellmann-Feynman forces by the chain rule (Observable response).

With an overlap S (nonorthogonal basis), FermiFreeEnergyOverlap takes the S
block values as a second input and hands back dF~/dS as well (Eq.
polynomial_response with dS != 0); a torch-built S(R) then adds the overlap term
of the forces.  Both gradients are the symmetric parts on the block pattern, as
H and S are symmetric.
"""

import torch


class FermiFreeEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values, engine, T, mu, n_terms):
        if values.dtype != torch.float64:
            raise TypeError("values must be float64")
        vals = values.detach().contiguous()
        engine.set_values(vals)
        grad = torch.empty_like(vals)
        out = engine.energy_and_dEdH(T, mu, n_terms, gradient=True, dFdH_out=grad)
        ctx.save_for_backward(grad)
        return torch.tensor(out["F"], dtype=torch.float64, device=values.device)

    @staticmethod
    def backward(ctx, grad_out):
        (grad,) = ctx.saved_tensors
        return grad_out * grad, None, None, None, None


class FermiFreeEnergyOverlap(torch.autograd.Function):
    @staticmethod
    def forward(ctx, h_values, s_values, engine, T, mu, n_terms, cg_tol):
        if h_values.dtype != torch.float64 or s_values.dtype != torch.float64:
            raise TypeError("values must be float64")
        h = h_values.detach().contiguous()
        # new H values drop the overlap: set S again after them
        engine.set_values(h)
        engine.set_overlap(s_values.detach().contiguous(), cg_tol=cg_tol)
        gh = torch.empty_like(h)
        out = engine.energy_and_dEdH(T, mu, n_terms, gradient=True, dFdH_out=gh)
        gs = torch.as_tensor(engine.dFdS(), dtype=torch.float64, device=h.device)
        ctx.save_for_backward(gh, gs)
        return torch.tensor(out["F"], dtype=torch.float64, device=h.device)

    @staticmethod
    def backward(ctx, grad_out):
        gh, gs = ctx.saved_tensors
        return grad_out * gh, grad_out * gs, None, None, None, None, None


def free_energy(values, engine, T, mu, n_terms, s_values=None, cg_tol=1e-13):
    """F~ as a differentiable function of the H block values (and of the S block
    values when s_values is given)."""
    if s_values is None:
        return FermiFreeEnergy.apply(values, engine, T, mu, n_terms)
    return FermiFreeEnergyOverlap.apply(values, s_values, engine, T, mu, n_terms, cg_tol)
