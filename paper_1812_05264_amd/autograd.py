"""torch.autograd.Function around the library's free-energy gradient.

FermiFreeEnergy.apply(values, engine, T, mu, n_terms) returns the probe estimate
F~ of tr g(H) for H with the engine's block pattern and the given block values;
its backward multiplies the incoming gradient by dF~/dH, which the library's
reverse-Clenshaw kernels produce in the forward call (paper: Analytical
free-energy derivatives).  Composing it with a torch-built H(R) gives
Hellmann-Feynman forces by the chain rule (Observable response).
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


def free_energy(values, engine, T, mu, n_terms):
    return FermiFreeEnergy.apply(values, engine, T, mu, n_terms)
