"""FD preconditioner parity on boxes with a different number of DOFs per
direction (the fused passes split planes and columns by direction, so square
planes would hide a swapped extent).  Reference: the oracle's FD application
(Section 3.3, the eigen-decomposition form of the Kronecker-product
preconditioner), element by element: FP64 max |d_i| <= 1e-12 max |ref_i|, FP32
<= 1e-5, BF16 operands <= 5e-2 (stated), also in place; non-uniform knots in one
case."""
import numpy as np
import pytest

import synth
from oracle.fd import FD
from oracle.wq import Space1D
from parity_gates import max_rel

pytestmark = pytest.mark.gpu


# the five after "nu" have extents a few DOFs past a multiple of 16 (a mostly
# empty last 16-block in every direction, as on the benchmark rings), M = 4..8;
# the last two have 4 DOFs (3 elements, the fewest fd_setup takes) in two or
# three directions (every block of those directions on the four-block 4 x 4 x 4
# product)
@pytest.mark.parametrize("els", [(5, 19, 40), (40, 19, 5), (70, 13, 30), (13, 97, 9), (9, 130, 17), "nu",
                                 (64, 66, 63), (80, 83, 82), (97, 96, 99), (113, 115, 112), (128, 131, 130),
                                 (3, 3, 3), (3, 14, 3)])
def test_fd_parity_box(els):
    import torch
    from paper_1712_08565_amd import wqfd
    p = 3
    if els == "nu":
        knots = [synth.nonuniform_knots(e, p, 400 + e) for e in (11, 37, 23)]
    else:
        knots = [synth.uniform_knots(e, p) for e in els]
    fd = FD([Space1D(k, p) for k in knots])
    P = wqfd.fd_setup(p, knots, wqfd.WQ_F64 | wqfd.WQ_F32 | wqfd.WQ_BF16)
    N = int(np.prod(P.n))
    r = synth.random_vector(N, 46)
    ref = fd.apply(r)
    print(f"[fd box] {els}: n = {P.n}", flush=True)
    x = torch.as_tensor(r, device="cuda")
    z = wqfd.fd_apply(P, x).cpu().numpy()
    z32 = wqfd.fd_apply(P, x.float(), prec=wqfd.WQ_F32).double().cpu().numpy()
    zbf = wqfd.fd_apply(P, x.float(), prec=wqfd.WQ_BF16).double().cpu().numpy()
    e = max_rel(z, ref)
    e32 = max_rel(z32, ref)
    ebf = max_rel(zbf, ref)
    print(f"[fd box] max entry error / max |ref|: fp64 {e:.2e}, fp32 {e32:.2e}, bf16 {ebf:.2e}")
    assert e <= 1e-12 and e32 <= 1e-5 and ebf <= 5e-2, (e, e32, ebf)
    wqfd.fd_apply(P, x, x)                                   # in place
    e_in = max_rel(x.cpu().numpy(), ref)
    assert e_in <= 1e-12, e_in
