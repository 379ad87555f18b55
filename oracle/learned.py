"""The learned step (oracle, float64).

Eq. 2: u_k = FV(u_{k-1}) + TC(u_{k-1}) when k is a multiple of the
correction interval k_c, else FV(u_{k-1}).

The flux block adds a learned correction to the physics stencil (Eq. 5,
O = O_P + O_L).  In per-cell form, with r_K the 16 raw network values of
kind K at a cell, the interpolation coefficients are
  c_K = c_P,K + r_K - mean(r_K)
which is the affine projection onto sum(c_K) = 1 around the physics stencil
(our reading of the sum-to-one constraint; r = 0 reduces the solver to the
plain FV solver, as Sec. 4.1 says of the physics-only model).

The network runs once per step on u_{k-1}; the same coefficients serve all
four RK sub-steps, and the temporal-correction field (channels 64, 65) comes
from the same forward pass.  The correction is applied as
u_k <- P(u_k + TC), so the state stays divergence-free.
"""
import torch

from . import fv
from .cnn import cnn_forward
from .projection import project
from .timestep import fv_step


def constrain(raw):
    """raw [B, 64, Ny, Nx] -> constrained coefficients c [B, 64, Ny, Nx]."""
    b, _, ny, nx = raw.shape
    r = raw.reshape(b, 4, 16, ny, nx)
    r = r - r.mean(dim=2, keepdim=True)
    cp = fv.plain_coefficients(raw.dtype).reshape(1, 4, 16, 1, 1)
    return (cp + r).reshape(b, 64, ny, nx)


def learned_fv_step(u, v, prm, weights, biases, step_index, bf16=False):
    """One learned step producing u_{step_index} from u_{step_index - 1}.
    Returns (u, v, net_out)."""
    x = torch.stack([u, v], dim=1)
    out = cnn_forward(x, weights, biases, bf16=bf16)
    coef = constrain(out[:, :64])
    un, vn = fv_step(u, v, prm, coef)
    kc = prm.get("k_c", 1)
    if kc > 0 and step_index % kc == 0:
        un, vn, _ = project(un + out[:, 64], vn + out[:, 65], prm)
    return un, vn, out


def learned_rollout(u, v, prm, weights, biases, nsteps, first_index=1, bf16=False):
    """States u_{first_index} .. u_{first_index + nsteps - 1}, stacked [T, B, Ny, Nx]."""
    us, vs = [], []
    for k in range(nsteps):
        u, v, _ = learned_fv_step(u, v, prm, weights, biases, first_index + k, bf16=bf16)
        us.append(u)
        vs.append(v)
    return torch.stack(us), torch.stack(vs)
