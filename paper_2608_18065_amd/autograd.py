"""log Psi(sigma; theta) as a torch.autograd.Function.

Forward: the recurrence of the library evaluates log Psi for given
configurations (Eqs. 2, 6, 8).  Backward: the library's reverse pass through
the recurrence forms the per-sample rows d log Psi / d theta and contracts
them with the incoming gradient (the vector-Jacobian product), so
``torch.autograd`` sees an exact gradient without tracing anything.

The output is real, shape (Ns, 2): column 0 is Re log Psi = 0.5 log P,
column 1 is Im log Psi (the phase).  Parameters are the flat FP64 vector of
the model's layout.
"""
import torch


class LogPsi(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, model, sigma):
        model.set_params(theta.detach())
        out = torch.view_as_real(model.logpsi(sigma)).clone()
        ctx.model = model
        ctx.save_for_backward(theta.detach(), sigma)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        theta, sigma = ctx.saved_tensors
        model = ctx.model
        model.set_params(theta)
        g = torch.view_as_complex(grad_out.to(torch.float64).contiguous())
        grad = model.logpsi_vjp(sigma, g)
        return grad, None, None


def log_psi(theta, model, sigma):
    """Differentiable (Ns, 2) real view of log Psi."""
    return LogPsi.apply(theta, model, sigma)
