"""fd_apply_noalloc: the FD preconditioner apply with the library's static
device scratch (for callers that cannot allocate) against fd_apply, which uses
the preconditioner's workspace.  Both run the same kernels, so the results must
agree bit for bit, in every prepared precision; the first call is on the larger
problem, the second on a smaller one (the scratch then holds the first call's
values).  The large-n path (n > 144, separate mode passes) and the size limit
are covered too.  FP64 is also checked against the oracle's FD inverse."""
import numpy as np
import pytest

import synth
from oracle.fd import FD
from oracle.wq import Space1D

pytestmark = pytest.mark.gpu


def _fd(n_el, p, mask):
    from paper_1712_08565_amd import wqfd
    k = synth.uniform_knots(n_el, p)
    print(f"[noalloc] fd_setup n_el={n_el} p={p} mask={mask}", flush=True)
    return wqfd.fd_setup(p, (k, k.copy(), k.copy()), mask), k


def _both(P, prec, seed):
    import torch
    from paper_1712_08565_amd import wqfd
    dt = torch.float64 if prec == wqfd.WQ_F64 else torch.float32
    r = torch.as_tensor(synth.random_vector(P.N, seed), device="cuda").to(dt)
    z_ref = wqfd.fd_apply(P, r, prec=prec)
    z = torch.full_like(r, float("nan"))
    wqfd.fd_apply_noalloc(P, r, z, prec=prec)
    torch.cuda.synchronize()
    return r, z, z_ref


def test_noalloc_fd_matches_fd_apply_large_then_small():
    import torch
    from paper_1712_08565_amd import wqfd
    mask = wqfd.WQ_F64 | wqfd.WQ_F32 | wqfd.WQ_BF16
    big, _ = _fd(64, 3, mask)              # N = 274,625 (the benchmark's p = 3 size)
    small, k_small = _fd(8, 4, mask)       # N = 1,000
    for P, label in ((big, "n_el=64 p=3"), (small, "n_el=8 p=4")):
        for prec in (wqfd.WQ_F64, wqfd.WQ_F32, wqfd.WQ_BF16):
            print(f"[noalloc] {label} prec={prec}", flush=True)
            r, z, z_ref = _both(P, prec, 60 + prec)
            d = float((z.double() - z_ref.double()).abs().max())
            assert bool(torch.isfinite(z).all()) and torch.equal(z, z_ref), (label, prec, d)
    # the smaller call against the oracle's FD inverse (FP64, 1e-12 relative)
    r, z, _ = _both(small, wqfd.WQ_F64, 61)
    ref = FD([Space1D(k_small, 4)] * 3).apply(r.cpu().numpy())
    e = float(np.linalg.norm(z.cpu().numpy() - ref) / np.linalg.norm(ref))
    print(f"[noalloc] n_el=8 p=4 vs oracle {e:.2e}", flush=True)
    assert e <= 1e-12, e


def test_noalloc_fd_large_n_path_and_alias():
    """n = 151 (> 144: the per-mode kernels), N = 3.44e6 (27.5 MB of FP64,
    inside the 32 MiB scratch); r and z may alias as in fd_apply."""
    import torch
    from paper_1712_08565_amd import wqfd
    P, _ = _fd(148, 5, wqfd.WQ_F64)
    assert P.N * 8 <= wqfd.WQ_FD_NOALLOC_BYTES
    r, z, z_ref = _both(P, wqfd.WQ_F64, 62)
    assert torch.equal(z, z_ref)
    x = r.clone()
    wqfd.fd_apply_noalloc(P, x, x)
    torch.cuda.synchronize()
    assert torch.equal(x, z_ref)


def test_noalloc_fd_rejects_sizes_beyond_the_scratch():
    import torch
    from paper_1712_08565_amd import wqfd
    from paper_1712_08565_amd._lib import WQ_ENOMEM
    P, _ = _fd(162, 3, wqfd.WQ_F32)        # n = 163, N = 4,330,747 > 32 MiB / 8
    assert P.N * 8 > wqfd.WQ_FD_NOALLOC_BYTES
    r = torch.zeros(P.N, dtype=torch.float32, device="cuda")
    z = torch.zeros_like(r)
    with pytest.raises(wqfd.WQError, match="static scratch") as ei:
        wqfd.fd_apply_noalloc(P, r, z)
    assert ei.value.code == WQ_ENOMEM
