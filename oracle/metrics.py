"""Down-sampling and evaluation metrics (oracle, float64).

Fine-to-coarse labels (Sec. 4.1: coarse flows are the fine flows down-sampled
in space and time; the operator is not specified).  Our reading, on the MAC
grid: face averaging, U[J, I] = (1/r) sum_{m<r} u[rJ + m, rI] and
V[J, I] = (1/r) sum_{m<r} v[rJ, rI + m].  The coarse divergence is then the
block mean of the fine divergence, so a divergence-free fine field stays
divergence-free.  Collocated fields use the block mean.

Vorticity at corners (i dx, j dy):
  w[j, i] = (v[j, i] - v[j, i-1]) / dx - (u[j, i] - u[j-1, i]) / dy.

Metrics (App. D.1, S32-S36): RMSE, MAE, MNAD, PCC and HCT.  Flow
statistics of a state: kinetic energy 1/2 <u^2 + v^2> and enstrophy
1/2 <w^2> (means over cells, per trajectory).  PCC is the
centred Pearson correlation per snapshot; HCT sums dt over snapshots whose PCC
exceeds a threshold (0.8 in the paper).
"""
import torch


def downsample_mac(u, v, r):
    ny, nx = u.shape[-2], u.shape[-1]
    uc = u[..., :, ::r].reshape(*u.shape[:-2], ny // r, r, nx // r).mean(dim=-2)
    vc = v[..., ::r, :].reshape(*v.shape[:-2], ny // r, nx // r, r).mean(dim=-1)
    return uc, vc


def downsample_collocated(q, r):
    ny, nx = q.shape[-2], q.shape[-1]
    return q.reshape(*q.shape[:-2], ny // r, r, nx // r, r).mean(dim=(-3, -1))


def vorticity(u, v, dx, dy):
    return (v - torch.roll(v, 1, dims=-1)) / dx - (u - torch.roll(u, 1, dims=-2)) / dy


def energy(u, v):
    """Kinetic energy per trajectory: 1/2 of the cell mean of u^2 + v^2."""
    return 0.5 * (u * u + v * v).mean(dim=(-2, -1))


def enstrophy(u, v, dx, dy):
    """Enstrophy per trajectory: 1/2 of the cell mean of the squared corner
    vorticity."""
    w = vorticity(u, v, dx, dy)
    return 0.5 * (w * w).mean(dim=(-2, -1))


def pcc(a, b):
    """Pearson correlation over the last two axes (S36)."""
    a = a - a.mean(dim=(-2, -1), keepdim=True)
    b = b - b.mean(dim=(-2, -1), keepdim=True)
    cov = (a * b).sum(dim=(-2, -1))
    return cov / torch.sqrt((a * a).sum(dim=(-2, -1)) * (b * b).sum(dim=(-2, -1)))


def rmse(pred, true):
    return torch.sqrt(((pred - true) ** 2).mean())


def mae(pred, true):
    return (pred - true).abs().mean()


def mnad(pred, true):
    """S34 for one trajectory: ||pred - true|| / (max(true) - min(true)), with
    the l2 norm taken per point over components and averaged over points."""
    return ((pred - true).abs().mean()) / (true.max() - true.min())


def hct(pcc_series, dt, threshold=0.8):
    return dt * float((pcc_series > threshold).sum())


def first_drop_time(pcc_series, dt, threshold=0.9):
    """Simulated time until the correlation first drops below threshold
    (snapshot k is at time (k+1) dt)."""
    below = (pcc_series < threshold).nonzero()
    if below.numel() == 0:
        return dt * pcc_series.numel()
    return dt * int(below[0].item())
