"""The coefficient network (oracle, float64).

The learnable part of the flux block (Sec. 3.4, Eqs. 5-7) is realised, in
the per-cell form this project builds, by a small convolutional network that
maps the coarse state (u, v) to 64 raw stencil values (4 kinds x 16 footprint
points) and a 2-channel temporal-correction field:

  conv 3x3, 2 -> 64, GELU;  4 x (conv 3x3, 64 -> 64, GELU);  conv 3x3, 64 -> 66

Every convolution is a cross-correlation with bias and periodic (circular)
padding of one cell (App. B.1, periodic BC padding).  GELU is the exact form
x * Phi(x) = x/2 (1 + erf(x / sqrt 2)).  The input channels are u and v as
stored on the MAC grid (the half-cell offset is not given to the network).

Weights are [Cout, Cin, 3, 3] (PyTorch order).  ``bf16=True`` rounds the
weights, the input and every hidden activation to bfloat16 (round to nearest
even), which is what a network stored in bfloat16 sees; accumulation stays in
float64.
"""
import math
import torch
import torch.nn.functional as F

LAYERS = [(2, 64), (64, 64), (64, 64), (64, 64), (64, 64), (64, 66)]


def gelu(x):
    return 0.5 * x * (1.0 + torch.erf(x / math.sqrt(2.0)))


def round_bf16(x):
    return x.to(torch.bfloat16).to(x.dtype)


def conv3x3_circular(x, w, b):
    """y[n, o, j, i] = b[o] + sum_{c, dy, dx} w[o, c, dy+1, dx+1] x[n, c, j+dy, i+dx]
    with periodic indices."""
    xp = F.pad(x, (1, 1, 1, 1), mode="circular")
    return F.conv2d(xp, w, b)


NCOEF = 64  # output channels 0..63: the 4 x 16 raw stencil values


def cnn_forward(x, weights, biases, bf16=False, return_acts=False):
    """x: [B, 2, Ny, Nx].  Returns [B, 66, Ny, Nx] (and the activations).

    bf16=True emulates the storage precision of a BF16 network: inputs,
    weights and every stored activation are rounded to bf16, and so are the
    64 stencil-coefficient outputs (they are stored like activations); the
    two temporal-correction outputs stay at full precision."""
    h = round_bf16(x) if bf16 else x
    acts = [h]
    nl = len(weights)
    for li in range(nl):
        w = round_bf16(weights[li]) if bf16 else weights[li]
        h = conv3x3_circular(h, w, biases[li])
        if li < nl - 1:
            h = gelu(h)
            if bf16:
                h = round_bf16(h)
        elif bf16:
            h = torch.cat([round_bf16(h[:, :NCOEF]), h[:, NCOEF:]], dim=1)
        acts.append(h)
    return (h, acts) if return_acts else h


def param_count():
    return sum(co * ci * 9 + co for ci, co in LAYERS)
