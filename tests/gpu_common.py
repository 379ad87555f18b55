"""Shared helpers for the GPU parity tests (HIP path through the C ABI vs the
FP64 CPU oracle)."""
import math
import sys

import torch

L = 2 * math.pi


def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2507_01975_amd import ldsv  # fails loudly if libldsv.so is missing
    return ldsv


def rel_l2(a, b):
    a = a.double().cpu()
    b = b.double().cpu()
    return ((a - b).norm() / b.norm().clamp_min(1e-300)).item()


def assert_fields_close(got, ref, rel=1e-5, elem=1e-5, what=""):
    """Relative L2 error <= rel, and every element within elem * max|ref|
    (so that an error confined to a few cells, such as a tile seam, cannot
    hide under the L2 norm of the whole field)."""
    e = rel_l2(got, ref)
    d = (got.double().cpu() - ref.double().cpu()).abs().max().item()
    m = ref.double().abs().max().item()
    assert e < rel and d <= elem * m, (what, e, d / max(m, 1e-300))


def dev(x, dtype):
    return x.to("cuda", dtype).contiguous()


def cpu64(x):
    return x.detach().double().cpu()


def announce(*a):
    """Print and flush the case before a GPU step, so a fault names it."""
    print("[gpu case]", *a, flush=True)
    sys.stdout.flush()


def oracle_prm(nx, ny, lx=L, ly=L, **kw):
    from oracle import fv
    return fv.grid_params(nx, ny, lx=lx, ly=ly, **kw)
