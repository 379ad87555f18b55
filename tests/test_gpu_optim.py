"""GPU parity of the training loss and the optimiser (Sec. 4.1 Eq. 13: MSE
of the unrolled rollout; App. D.3: Adam) through the C ABI against the FP64
oracle, element by element."""
import pytest
import torch

from oracle import optim
from tests.gpu_common import announce, cpu64, dev, need_gpu

pytestmark = pytest.mark.gpu

EPS32 = 2.0 ** -24


@pytest.mark.parametrize("nx,ny,b,scale", [(16, 8, 3, 0.7), (64, 64, 2, 1.0), (8, 8, 1, 1e-3)])
def test_mse_grad_matches_oracle(nx, ny, b, scale):
    L_ = need_gpu()
    announce("mse_grad", nx, ny, b, scale)
    g = torch.Generator().manual_seed(nx + ny + b)
    u, v, lu, lv = (torch.randn(b, ny, nx, generator=g, dtype=torch.float64).float().double()
                    for _ in range(4))
    s = L_.Solver(nx, ny, b)
    loss = torch.full((1,), 0.25, dtype=torch.float64, device="cuda")  # accumulated into
    gu, gv = s.mse_grad(dev(u, torch.float32), dev(v, torch.float32), dev(lu, torch.float32),
                        dev(lv, torch.float32), scale=scale, loss=loss)
    # loss: FP64 reduction of the FP32 inputs, added to the buffer's value
    ua = u.clone().requires_grad_(True)
    va = v.clone().requires_grad_(True)
    ref = scale * optim.mse_loss(ua, va, lu, lv)
    ref.backward()
    assert loss.item() == pytest.approx(0.25 + ref.item(), rel=1e-12)
    # gradient scale (u - lu) / n: one FP32 subtraction and one FP32 product
    for got, want in ((gu, ua.grad), (gv, va.grad)):
        d = (cpu64(got) - want).abs()
        assert (d <= 4 * EPS32 * want.abs() + 1e-30).all(), d.max().item()
    # without a loss buffer only the gradient is written; without gradients
    # only the loss
    gu2, _ = s.mse_grad(dev(u, torch.float32), dev(v, torch.float32), dev(lu, torch.float32),
                        dev(lv, torch.float32), scale=scale)
    assert torch.equal(gu2, gu)
    loss2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    s.mse_grad(dev(u, torch.float32), dev(v, torch.float32), dev(lu, torch.float32),
               dev(lv, torch.float32), scale=scale, loss=loss2, want_grad=False)
    assert loss2.item() == pytest.approx(ref.item(), rel=1e-12)


@pytest.mark.parametrize("n", [1, 1000, 187010])
def test_adam_steps_match_oracle(n):
    """Five Adam steps (bias correction at t = 1..5) with a fresh gradient per
    step, against the oracle's update in FP64 from the same FP32 values;
    187,010 is the coefficient network's parameter count."""
    L_ = need_gpu()
    announce("adam", n)
    g = torch.Generator().manual_seed(n)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    w = torch.randn(n, generator=g, dtype=torch.float64).float()
    m = torch.zeros(n, dtype=torch.float32)
    v = torch.zeros(n, dtype=torch.float32)
    wd, md, vd = w.cuda(), m.cuda(), v.cuda()
    wr, mr, vr = w.double(), m.double(), v.double()
    ma = torch.zeros(n, dtype=torch.float64)     # envelope of |m| without cancellation
    for t in range(1, 6):
        gr = torch.randn(n, generator=g, dtype=torch.float64) * 10.0 ** torch.randint(
            -4, 2, (n,), generator=g).double()
        if n > 1:
            gr[0] = 0.0                       # m = v = 0 there: the update is 0 / (0 + eps)
        gr = gr.float()
        L_.adam_step(wd, gr.cuda(), md, vd, t, lr, b1, b2, eps)
        wr, mr, vr = optim.adam_step(wr, gr.double(), mr, vr, t, lr=lr, b1=b1, b2=b2, eps=eps)
        ma = b1 * ma + (1 - b1) * gr.double().abs()
        torch.cuda.synchronize()
        # moments: a few FP32 roundings per step of the running sums.  The
        # first moment is a signed sum: its rounding errors scale with the
        # sum of the magnitudes of its terms (ma), not with |m|, which can
        # cancel; the second moment has no cancellation
        assert ((cpu64(md) - mr).abs() <= 4 * t * EPS32 * ma).all(), t
        assert ((cpu64(vd) - vr).abs() <= 4 * t * EPS32 * (vr.abs() + gr.double() ** 2)).all(), t
        # weights: one FP32 rounding of w per step (the oracle keeps FP64)
        # plus a relative error of a few ulps in each update, whose size is
        # at most about lr
        dw = (cpu64(wd) - wr).abs()
        assert (dw <= (t + 1) * EPS32 * wr.abs() + 1e-5 * lr * t).all(), (t, dw.max().item())
    if n > 1:
        assert cpu64(wd)[0].item() == w[0].item()   # zero gradient every step: no move
