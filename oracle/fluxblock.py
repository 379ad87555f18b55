"""The flux-block model step (oracle, float64): the paper's own learnable
flux block (Sec. 3.4, Eqs. 5-8) inside the RK4 + projection FV module.

TEST INFRASTRUCTURE ONLY (see the package header).

Every interpolated face value and every face derivative of the momentum
residual is O^(m) = O_P^(m) + O_L^(m) + O_F^(m), m in {i, d}:
  O_P  the physics kernels (midpoint average; the fourth-order derivative),
  O_L  spatially uniform learnable 5x4 kernels, one per kind and per m
       (each component keeps its own parameters: nothing is shared between
       the kinds or between m = i and m = d),
  O_F  one FNO per m mapping the state (u, v) to 4 fields, one per kind
       (fno module).
The FNOs run once per step on the step's input state and their fields are
held fixed over the four RK sub-steps, the same reading as for the per-cell
network.  Parameters: dict(wi [4, 20], wd [4, 20], fno_i, fno_d), where
either FNO may be None (then O_F^(m) = 0).

The temporal correction block (Eq. 2; Sec. 3.5 and the error-propagation
argument of its appendix): every k_c steps the states since the last
correction, u_{k-k_c} .. u_{k-1}, go through an FNO (params["tc"]: input
planes (u, v) of each state, oldest first; 2 outputs) whose output is added
to the FV update: u_k = P(FV(u_{k-1}) + TC).  The projection keeps the
corrected state divergence-free (P is linear and P FV(u) = FV(u), so this
equals FV(u_{k-1}) + P TC).
"""
import torch

from . import fno
from .projection import project
from .timestep import fv_step


def flux_record(u, v, params):
    """The flux-block record (wi, wd, fi, fd) for the state (u, v)."""
    x = torch.stack([u, v], dim=1)
    fi = fno.fno_forward(x, params["fno_i"]) if params.get("fno_i") is not None else None
    fd = fno.fno_forward(x, params["fno_d"]) if params.get("fno_d") is not None else None
    return {"wi": params.get("wi"), "wd": params.get("wd"), "fi": fi, "fd": fd}


def fluxblock_step(u, v, prm, params):
    """One step u_k -> u_{k+1} of the FV module with the flux block."""
    return fv_step(u, v, prm, flux=flux_record(u, v, params))


def fluxblock_rollout(u, v, prm, params, nsteps):
    """States u_1 .. u_nsteps, stacked [T, B, Ny, Nx]."""
    us, vs = [], []
    for _ in range(nsteps):
        u, v = fluxblock_step(u, v, prm, params)
        us.append(u)
        vs.append(v)
    return torch.stack(us), torch.stack(vs)


def tc_input(hist_u, hist_v):
    """[B, 2 k_c, Ny, Nx]: planes (u_j, v_j) of the history, oldest first."""
    planes = []
    for u, v in zip(hist_u, hist_v):
        planes += [u, v]
    return torch.stack(planes, dim=1)


def model_step(hist_u, hist_v, prm, params, step_index):
    """u_k from the history u_{k-k_c} .. u_{k-1} (lists, oldest first; only
    the last is read unless the correction applies at k = step_index)."""
    u, v = fluxblock_step(hist_u[-1], hist_v[-1], prm, params)
    kc = prm.get("k_c", 1)
    tc = params.get("tc")
    if tc is not None and step_index % kc == 0:
        d = fno.fno_forward(tc_input(hist_u[-kc:], hist_v[-kc:]), tc)
        u, v, _ = project(u + d[:, 0], v + d[:, 1], prm)
    return u, v


def model_rollout(u0, v0, prm, params, nsteps):
    """States u_1 .. u_nsteps of the complete model (flux block + temporal
    correction), stacked [T, B, Ny, Nx]."""
    hu, hv = [u0], [v0]
    for k in range(1, nsteps + 1):
        u, v = model_step(hu, hv, prm, params, k)
        hu.append(u)
        hv.append(v)
    return torch.stack(hu[1:]), torch.stack(hv[1:])
