"""FD preconditioner parity on boxes with a different number of DOFs per
direction (the fused passes split planes and columns by direction, so square
planes would hide a swapped extent).  Reference: the oracle's FD application
(Section 3.3, the eigen-decomposition form of the Kronecker-product
preconditioner), FP64 to 1e-12 relative, FP32 to 1e-5, also in place."""
import numpy as np
import pytest

import synth
from oracle.fd import FD
from oracle.wq import Space1D

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("els", [(5, 19, 40), (40, 19, 5), (70, 13, 30), (13, 97, 9), (9, 130, 17)])
def test_fd_parity_box(els):
    import torch
    from paper_1712_08565_amd import wqfd
    p = 3
    knots = [synth.uniform_knots(e, p) for e in els]
    fd = FD([Space1D(k, p) for k in knots])
    P = wqfd.fd_setup(p, knots, wqfd.WQ_F64 | wqfd.WQ_F32)
    N = int(np.prod(P.n))
    r = synth.random_vector(N, 46)
    ref = fd.apply(r)
    print(f"[fd box] elements {els}: n = {P.n}", flush=True)
    x = torch.as_tensor(r, device="cuda")
    z = wqfd.fd_apply(P, x).cpu().numpy()
    z32 = wqfd.fd_apply(P, x.float(), prec=wqfd.WQ_F32).double().cpu().numpy()
    e = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    e32 = np.linalg.norm(z32 - ref) / np.linalg.norm(ref)
    assert e <= 1e-12 and e32 <= 1e-5, (e, e32)
    wqfd.fd_apply(P, x, x)                                   # in place
    e_in = np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert e_in <= 1e-12, e_in
