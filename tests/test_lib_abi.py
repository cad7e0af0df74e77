"""The C ABI library loads without a GPU and exports every function that
include/wqfd.h declares; host-side argument errors are reported as documented
(no device work is started by these calls)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wqfd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][A-Za-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if not n.startswith("__")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("wq_setup", "wq_apply", "wq_apply_T", "fd_setup", "fd_apply", "krylov_solve", "ir_solve",
              "wq_grad_K", "wq_grad_f", "wq_rhs"):
        assert n in names


def test_library_loads_and_exports_every_declared_symbol():
    from paper_1712_08565_amd import _lib
    L = _lib.lib()
    declared = declared_functions()
    bound = {n for n, _, _ in _lib.SIGNATURES}
    assert set(declared) == bound, (set(declared) ^ bound)
    for n in declared:
        assert hasattr(L, n)
    assert b"gfx950" in L.wq_version()


def test_noalloc_entry_checks_arguments_on_the_host():
    """fd_apply_noalloc refuses a null handle or vector before any device work,
    and the binding's scratch limit is the header's."""
    from paper_1712_08565_amd import _lib
    L = _lib.lib()
    assert L.fd_apply_noalloc(None, _lib.WQ_F64, None, None, None) == _lib.WQ_EINVAL
    assert len(L.wq_last_error()) > 0
    assert L.wq_alpha_mean(None, C.byref(C.c_double()), None) == _lib.WQ_EINVAL
    m = re.search(r"#define\s+WQ_FD_NOALLOC_BYTES\s+\((\d+)u\s*<<\s*(\d+)\)", open(HEADER).read())
    assert m and int(m.group(1)) << int(m.group(2)) == _lib.WQ_FD_NOALLOC_BYTES


def _setup_args(p, knots):
    ks = [np.ascontiguousarray(k, dtype=np.float64) for k in knots]
    nk = (C.c_int32 * 3)(*[len(k) for k in ks])
    kp = (C.c_void_p * 3)(*[k.ctypes.data for k in ks])
    return ks, nk, kp


@pytest.mark.parametrize("case", ["p_low", "p_high", "not_open", "multiple_knot", "too_few_elements"])
def test_invalid_spaces_are_rejected_on_the_host(case):
    from paper_1712_08565_amd import _lib
    L = _lib.lib()
    p = 3
    k = synth.uniform_knots(6, p)
    if case == "p_low":
        p = 1
    elif case == "p_high":
        p = 11
    elif case == "not_open":
        k = k.copy()
        k[0] = -0.1
    elif case == "multiple_knot":
        k = k.copy()
        k[p + 2] = k[p + 1]
    elif case == "too_few_elements":
        k = synth.uniform_knots(2, p)
    ks, nk, kp = _setup_args(p, (k, k, k))
    m = len(k) - 3 - 1
    ctrl = np.zeros((m, m, m, 3))
    need = C.c_size_t(0)
    rc = L.wq_setup(p, nk, kp, C.c_void_p(ctrl.ctypes.data), 0, None, 1, None, 0, C.byref(need), None, None)
    assert rc == _lib.WQ_EINVAL
    assert len(L.wq_last_error()) > 0
    rc = L.fd_setup(p, nk, kp, 1, None, 0, C.byref(need), None, None)
    assert rc == _lib.WQ_EINVAL


def test_size_query_needs_no_device():
    from paper_1712_08565_amd import _lib
    L = _lib.lib()
    wl = synth.workload("cube12_p3")
    ks, nk, kp = _setup_args(wl.p, wl.knots())
    ctrl = wl.ctrl()
    need = C.c_size_t(0)
    assert L.wq_setup(3, nk, kp, C.c_void_p(ctrl.ctypes.data), 0, None, 3, None, 0, C.byref(need), None,
                      None) == 0
    Nq = 31 ** 3
    assert need.value > (10 + 3 + 6) * 8 * Nq + 6 * 4 * Nq
    assert L.fd_setup(3, nk, kp, 7, None, 0, C.byref(need), None, None) == 0
    assert need.value >= 3 * 13 * 13 * 8 + 13 ** 3 * 8
    # bad enums are rejected before any device work
    assert L.wq_setup(3, nk, kp, C.c_void_p(ctrl.ctypes.data), 5, None, 1, None, 0, C.byref(need), None,
                      None) == _lib.WQ_EINVAL
    assert L.wq_setup(3, nk, kp, C.c_void_p(ctrl.ctypes.data), 0, None, 8, None, 0, C.byref(need), None,
                      None) == _lib.WQ_EINVAL


def test_small_or_misaligned_workspace_is_refused():
    """WQ_ENOMEM for a workspace below the size query, WQ_EINVAL for one that is
    not 256-byte aligned; both are decided before the workspace is touched (the
    stand-in address below is never dereferenced)."""
    from paper_1712_08565_amd import _lib
    L = _lib.lib()
    wl = synth.workload("cube5_p2")
    ks, nk, kp = _setup_args(wl.p, wl.knots())
    ctrl = wl.ctrl()
    need = C.c_size_t(0)
    h = C.c_void_p(0)
    assert L.wq_setup(wl.p, nk, kp, C.c_void_p(ctrl.ctypes.data), 0, None, 1, None, 0, C.byref(need), None,
                      None) == 0
    fake = 1 << 30
    assert L.wq_setup(wl.p, nk, kp, C.c_void_p(ctrl.ctypes.data), 0, None, 1, C.c_void_p(fake), need.value - 1,
                      None, None, C.byref(h)) == _lib.WQ_ENOMEM
    assert L.wq_setup(wl.p, nk, kp, C.c_void_p(ctrl.ctypes.data), 0, None, 1, C.c_void_p(fake + 8), need.value,
                      None, None, C.byref(h)) == _lib.WQ_EINVAL
    assert L.fd_setup(wl.p, nk, kp, 1, None, 0, C.byref(need), None, None) == 0
    assert L.fd_setup(wl.p, nk, kp, 1, C.c_void_p(fake), need.value - 1, None, None, C.byref(h)) == _lib.WQ_ENOMEM
    assert L.fd_setup(wl.p, nk, kp, 1, C.c_void_p(fake + 8), need.value, None, None, C.byref(h)) == _lib.WQ_EINVAL
    assert not h.value


def test_memory_is_order_N_independent_of_p():
    """The operator's memory is a fixed number of bytes per quadrature point
    (one figure for the fused kernels, p <= 7, a larger one for the staged
    kernels, p >= 8) and does not grow with p per degree of freedom (the memory claims of Sections
    3.1-3.2), while an assembled matrix would need about 12 (2p+1)^3 bytes per
    degree of freedom."""
    from paper_1712_08565_amd import _lib
    L = _lib.lib()
    per_point, per_dof = [], []
    for p in range(2, 11):
        k = synth.uniform_knots(16, p)
        ks, nk, kp = _setup_args(p, (k, k, k))
        ctrl = synth.control_net("identity", (k, k, k), p)
        need = C.c_size_t(0)
        assert L.wq_setup(p, nk, kp, C.c_void_p(ctrl.ctypes.data), 0, None, 1, None, 0, C.byref(need), None,
                          None) == 0
        n, nq = 16 + p - 2, 2 * 16 + 2 * p + 1
        per_point.append(need.value / nq ** 3)
        per_dof.append(need.value / n ** 3)
    # two regimes, each a fixed number of bytes per point: p <= 7 (fused kernels; the
    # gradient needs no N_q-sized fields) and p >= 8 (staged kernels and gradient)
    fused, staged = per_point[:6], per_point[6:]
    assert max(fused) / min(fused) < 1.02 and max(staged) / min(staged) < 1.02, per_point
    assert max(per_point) / min(per_point) < 1.5, per_point
    assert max(per_dof[1:6]) <= per_dof[0] and max(per_dof[7:]) <= per_dof[6], per_dof   # no growth with p
    assert per_dof[-1] < 0.05 * 12 * 21 ** 3                 # 2.6% of an assembled matrix at p = 10


def test_binding_checks_sizes_before_any_device_work():
    """The torch binding refuses arguments whose size the C ABI cannot check (plain
    pointers whose extent follows from the operator): a control net of the wrong
    size, a conductivity field of the wrong length or on the host, an unknown
    k_kind and a workspace that is host memory.  All are ValueErrors raised before
    the library is called."""
    import types

    import torch

    from paper_1712_08565_amd import wqfd
    wl = synth.workload("cube12_p3")
    ctrl = wl.ctrl()
    with pytest.raises(ValueError, match="ctrl"):
        wqfd.wq_setup(wl.p, wl.knots(), ctrl[:-1], device="cpu")
    with pytest.raises(ValueError, match="k_kind"):
        wqfd.wq_setup(wl.p, wl.knots(), ctrl, k_kind=5, device="cpu")
    with pytest.raises(ValueError, match="K_q is required"):
        wqfd.wq_setup(wl.p, wl.knots(), ctrl, k_kind=wqfd.WQ_K_SCALAR, device="cpu")
    op = types.SimpleNamespace(Nq=40, N=8, handle=None, device="cpu")
    with pytest.raises(ValueError, match="K_q"):
        wqfd.wq_set_coef(op, wqfd.WQ_K_SCALAR, torch.zeros(40, dtype=torch.float64))     # host memory
    with pytest.raises(ValueError, match="k_kind"):
        wqfd.wq_set_coef(op, 2, None)
    with pytest.raises(ValueError, match="K_q is required"):
        wqfd.wq_set_coef(op, wqfd.WQ_K_SYM6, None)
    with pytest.raises(ValueError, match="ws"):
        wqfd._ws_bytes(torch.zeros(64, dtype=torch.uint8), 16, "ws")


def test_new_entries_check_arguments_on_the_host():
    """wq_setup_nurbs, wq_grad_Kf and the Gauss-point evaluator refuse null and
    out-of-range arguments before any device work; the evaluator's size query
    needs no device and grows with the control net (32 bytes per point) and the
    Gauss tables."""
    from paper_1712_08565_amd import _lib
    L = _lib.lib()
    wl = synth.workload("nurbs8_p3")
    ks, nk, kp = _setup_args(wl.p, wl.knots())
    ctrl, w = wl.ctrl(), wl.weights()
    need = C.c_size_t(0)
    assert L.wq_setup_nurbs(wl.p, nk, kp, C.c_void_p(ctrl.ctypes.data), None, 0, None, 1, None, 0,
                            C.byref(need), None, None) == _lib.WQ_EINVAL
    assert L.wq_setup_nurbs(wl.p, nk, kp, C.c_void_p(ctrl.ctypes.data), C.c_void_p(w.ctypes.data), 0, None, 1,
                            None, 0, C.byref(need), None, None) == 0 and need.value > 0
    assert L.wq_grad_Kf(None, None, None, None, None, None) == _lib.WQ_EINVAL
    for ng in (0, 33):
        assert L.wq_eval_setup(wl.p, nk, kp, C.c_void_p(ctrl.ctypes.data), None, ng, None, 0, C.byref(need), None,
                               None) == _lib.WQ_EINVAL
    sizes = []
    for ng in (4, 6):
        assert L.wq_eval_setup(wl.p, nk, kp, C.c_void_p(ctrl.ctypes.data), C.c_void_p(w.ctypes.data), ng, None, 0,
                               C.byref(need), None, None) == 0
        sizes.append(need.value)
    assert sizes[0] >= ctrl[..., 0].size * 32 and sizes[1] > sizes[0]
    assert L.wq_eval_slab(None, None, 0, 1, None, None, None, None, None) == _lib.WQ_EINVAL
    assert L.wq_eval_dims(None, None, None) == _lib.WQ_EINVAL
