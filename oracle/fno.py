"""Fourier neural operator (oracle, float64): the frequency-domain part O_F
of the flux block (Sec. 3.4, Eq. 8; the FNO description in the appendix on
baseline models; Li et al., ICLR 2021).

TEST INFRASTRUCTURE ONLY (see the package header).

  v_0     = P x + b_P                          pointwise lift, n_in -> width
  v_{l+1} = sigma(K_l v_l + W_l v_l + b_l)     l = 0 .. L-1
  out     = Q v_L + b_Q                        pointwise projection, width -> n_out

sigma is the exact-erf GELU after every Fourier layer except the last one
(the layer stack of Li et al.'s two-dimensional FNO); the projection Q is a
single pointwise linear map (the paper only calls Q a learnable projection).

The spectral convolution K keeps a band of modes of the real 2D transform:
  V_i(k)  = sum_{y,x} v_i[y, x] exp(-2 pi i (k_y y / N_y + k_x x / N_x)),
            0 <= k_x <= N_x / 2
  Y_o(k)  = sum_i R[r(k_y), k_x, i, o] V_i(k)   for k_y in [0, M_y) U [N_y - M_y, N_y)
            and k_x < M_x; Y = 0 elsewhere (r numbers the retained rows:
            r = k_y below M_y, r = k_y - N_y + 2 M_y above)
  (K v)_o[y, x] = (1 / (N_x N_y)) sum_{k_y} sum_{k_x = 0}^{N_x/2} w(k_x)
                  Re(Y_o(k) exp(2 pi i (k_y y / N_y + k_x x / N_x)))
with w = 1 at k_x = 0 and k_x = N_x / 2 and w = 2 otherwise: the real
inverse transform of a half spectrum, which reads only the real part of the
k_x = 0 and Nyquist columns.  This is what torch.fft.rfft2 / irfft2 compute
(Li et al.'s implementation); the brute-force test writes the sums out.

Parameters: dict(P_w [width, n_in], P_b [width], layers = [dict(R complex
[2 M_y, M_x, width, width] (retained row, k_x, in, out), W [width, width]
(out, in), b [width])], Q_w [n_out, width], Q_b [n_out]).
"""
import torch

from .cnn import gelu


def retained_rows(ny, my):
    """Row wavenumbers k_y kept by a spectral convolution, in retained-row order."""
    assert 2 * my <= ny
    return list(range(my)) + list(range(ny - my, ny))


def spectral_conv(v, R):
    """v [B, C, Ny, Nx] real; R complex [2 My, Mx, C, Cout] -> [B, Cout, Ny, Nx]."""
    b, c, ny, nx = v.shape
    two_my, mx = R.shape[0], R.shape[1]
    assert mx <= nx // 2 + 1
    rows = retained_rows(ny, two_my // 2)
    V = torch.fft.rfft2(v)                               # [B, C, Ny, Nx/2 + 1]
    Vk = V[:, :, rows, :mx]                              # [B, C, 2My, Mx]
    Yk = torch.einsum("bcrk,rkco->bork", Vk, R)
    Y = torch.zeros(b, R.shape[3], ny, nx // 2 + 1, dtype=V.dtype)
    Y[:, :, rows, :mx] = Yk
    return torch.fft.irfft2(Y, s=(ny, nx))


def pointwise(v, w, bias):
    """out[b, o, y, x] = sum_i w[o, i] v[b, i, y, x] + bias[o]."""
    return torch.einsum("oi,biyx->boyx", w, v) + bias.view(1, -1, 1, 1)


def fno_forward(x, p, return_acts=False):
    """x [B, n_in, Ny, Nx] -> [B, n_out, Ny, Nx] (and the layer pre-activations)."""
    h = pointwise(x, p["P_w"], p["P_b"])
    acts = [h]
    nl = len(p["layers"])
    for li, lay in enumerate(p["layers"]):
        z = spectral_conv(h, lay["R"]) + pointwise(h, lay["W"], lay["b"])
        h = gelu(z) if li < nl - 1 else z
        acts.append(h)
    out = pointwise(h, p["Q_w"], p["Q_b"])
    return (out, acts) if return_acts else out


def from_arrays(a):
    """FNO parameters from the real arrays of synthetic_inputs.fno_weights
    (float64 tensors; R assembled from its real and imaginary parts)."""
    t = lambda z: torch.as_tensor(z, dtype=torch.float64)
    return {
        "P_w": t(a["P_w"]), "P_b": t(a["P_b"]),
        "layers": [{"R": torch.complex(t(l["R_re"]), t(l["R_im"])), "W": t(l["W"]),
                    "b": t(l["b"])} for l in a["layers"]],
        "Q_w": t(a["Q_w"]), "Q_b": t(a["Q_b"]),
    }


def param_count(width, layers, modes, n_in=2, n_out=4):
    """Real parameters of one FNO (a complex weight counts twice)."""
    per_layer = 2 * (2 * modes * modes * width * width) + width * width + width
    return width * n_in + width + layers * per_layer + n_out * width + n_out
