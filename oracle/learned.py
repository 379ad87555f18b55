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

Learned derivative stencils (the m = d operator in per-cell form): a second
network of the same layer shapes (the paper keeps separate parameters for
m = i and m = d, nothing shared) gives 64 raw values r per cell (its two
last outputs are not used).  With x_s = a_s - 1/2 the position of footprint
point s along the face normal and b_s its position across (units of the
spacings), the derivative weights are
  w_K = w_P,K + r_K - mean(r_K) - x (x . r_K) / (x . x) - b (b . r_K) / (b . b)
the affine projection, around the fourth-order kernel w_P, onto the weights
with sum(w) = 0, sum(w x) = 1 and sum(w b) = 0: zero derivative of a
constant and the exact normal derivative of every linear field (our reading
of the derivative analogue of the sum-to-one constraint; without the
across moment a tangential gradient would leak into the face derivative with
a weight that does not shrink with the spacing).  Over the footprint x and b
have mean zero, x . b = 0, x . x = 16 and b . b = 24, so the three
constraint directions are orthogonal and the projection takes this form.
r = 0 gives back the fourth-order kernel.

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


NORMAL_X = torch.tensor([a - 0.5 for a, _ in fv.FOOTPRINT], dtype=torch.float64)
ACROSS_B = torch.tensor([float(b) for _, b in fv.FOOTPRINT], dtype=torch.float64)


def constrain_deriv(raw):
    """raw [B, 64, Ny, Nx] -> derivative weights w [B, 64, Ny, Nx] (units 1/h)."""
    b, _, ny, nx = raw.shape
    r = raw.reshape(b, 4, 16, ny, nx)
    x = NORMAL_X.to(raw.dtype).reshape(1, 1, 16, 1, 1)
    y = ACROSS_B.to(raw.dtype).reshape(1, 1, 16, 1, 1)
    r = (r - r.mean(dim=2, keepdim=True) - x * (x * r).sum(dim=2, keepdim=True) / (x * x).sum()
         - y * (y * r).sum(dim=2, keepdim=True) / (y * y).sum())
    wp = fv.plain_deriv_coefficients(raw.dtype).reshape(1, 4, 16, 1, 1)
    return (wp + r).reshape(b, 64, ny, nx)


def learned_fv_step(u, v, prm, weights, biases, step_index, bf16=False, dnet=None):
    """One learned step producing u_{step_index} from u_{step_index - 1}.
    dnet: optional (weights, biases) of the derivative-stencil network.
    Returns (u, v, net_out)."""
    x = torch.stack([u, v], dim=1)
    out = cnn_forward(x, weights, biases, bf16=bf16)
    coef = constrain(out[:, :64])
    dcoef = None
    if dnet is not None:
        dcoef = constrain_deriv(cnn_forward(x, dnet[0], dnet[1], bf16=bf16)[:, :64])
    un, vn = fv_step(u, v, prm, coef, dcoef=dcoef)
    kc = prm.get("k_c", 1)
    if kc > 0 and step_index % kc == 0:
        un, vn, _ = project(un + out[:, 64], vn + out[:, 65], prm)
    return un, vn, out


def learned_rollout(u, v, prm, weights, biases, nsteps, first_index=1, bf16=False, dnet=None):
    """States u_{first_index} .. u_{first_index + nsteps - 1}, stacked [T, B, Ny, Nx]."""
    us, vs = [], []
    for k in range(nsteps):
        u, v, _ = learned_fv_step(u, v, prm, weights, biases, first_index + k, bf16=bf16,
                                  dnet=dnet)
        us.append(u)
        vs.append(v)
    return torch.stack(us), torch.stack(vs)
