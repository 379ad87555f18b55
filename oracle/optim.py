"""Training loss and optimiser (oracle, float64).

Loss (Sec. 4.1, Eq. 13): the mean over samples of the MSE between the
autoregressive rollout and the labels.  Optimiser: Adam (Kingma and Ba,
2015) with the paper's learning rate 1e-4 (App. D.3) and the usual
beta1 = 0.9, beta2 = 0.999, eps = 1e-8 (unstated in the paper):
  m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
  w -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
"""
import torch


def mse_loss(pred_u, pred_v, lab_u, lab_v):
    return 0.5 * (((pred_u - lab_u) ** 2).mean() + ((pred_v - lab_v) ** 2).mean())


def adam_step(w, g, m, v, t, lr=1e-4, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (torch.sqrt(vh) + eps), m, v
