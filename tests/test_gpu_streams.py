"""Library calls on a torch stream other than the current one.  The binding
orders such a call after the work already queued on the current stream (where
its inputs were produced) and keeps a workspace it allocates itself alive until
the side stream's queued work is done (a solve can return with a speculative
half-iteration still queued).  Results on the side stream equal those on the
current stream to rounding (the applies add with atomics)."""
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_solves_and_apply_on_a_side_stream():
    import torch
    from paper_1712_08565_amd import problem, wqfd
    wl = synth.workload("ring8_p3")
    print("[streams] setup ring8_p3", flush=True)
    dp = problem.build(wl, wqfd.WQ_F64 | wqfd.WQ_F32, wqfd.WQ_F64 | wqfd.WQ_F32)
    x0, it0, _ = wqfd.krylov_solve(dp.A, dp.P, dp.b, rtol=1e-12)
    xm0, _, _, _ = wqfd.ir_solve(dp.A, dp.P, dp.b, fd_prec=wqfd.WQ_F32, rtol=1e-12, tau_inner=1e-4)
    w0 = wqfd.wq_apply(dp.A, x0)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    for rep in range(3):
        # inputs produced on the current stream right before each call
        b = dp.b * 1.0
        v = x0 * 1.0
        x, it, rel = wqfd.krylov_solve(dp.A, dp.P, b, rtol=1e-12, stream=side)
        xm, _, _, relm = wqfd.ir_solve(dp.A, dp.P, b, fd_prec=wqfd.WQ_F32, rtol=1e-12, tau_inner=1e-4,
                                       stream=side)
        w = wqfd.wq_apply(dp.A, v, stream=side)
        side.synchronize()
        print(f"[streams] rep {rep}: {it} iterations (current stream {it0}), relres {rel:.1e} / {relm:.1e}",
              flush=True)
        assert rel <= 1e-12 and relm <= 1e-12
        assert torch.linalg.norm(x - x0).item() <= 1e-9 * torch.linalg.norm(x0).item()
        assert torch.linalg.norm(xm - xm0).item() <= 1e-9 * torch.linalg.norm(xm0).item()
        assert torch.max(torch.abs(w - w0)).item() <= 1e-12 * torch.max(torch.abs(w0)).item()
