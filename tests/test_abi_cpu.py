"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function the header declares, and the workspace planner and argument
checks behave."""
import ctypes

import pytest

import paper_2505_00494_amd as P
from paper_2505_00494_amd import qrctm as B


def test_library_exports_every_declared_function():
    L = P.lib()
    names = P.header_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert missing == []


def test_default_opts():
    o = B.default_opts()
    assert o.precision == B.PREC_FP64 and o.n_warmup == -1 and o.k_tracked == -1
    assert o.qr_sing_tol == 1e-14 and o.mixed_tol == 1e-6
    assert o.edge_split == 1 and o.grad_mode == B.GRAD_CHECKPOINT
    assert o.fp_tol == 1e-10 and o.fp_max_iter == 1000
    assert o.grad_keep_yz == 0 and o.qr_reg_eps == 0.0


def test_default_tracked_steps_per_bond_dimension():
    # k_tracked = -1 plans the checkpoints of the per-D choice of the paper's
    # timing study (Fig. 3 caption: 10, 12, 14, 16, 20, 24 for D = 2..7; 28 at D = 8)
    L = P.lib()
    auto = B.default_opts()
    for D, k in [(2, 10), (3, 12), (4, 14), (5, 16), (6, 20), (7, 24), (8, 28)]:
        chi = D * D
        fixed = B.default_opts(k_tracked=k)
        assert (L.ctm_workspace_bytes(2, D, chi, ctypes.byref(auto))
                == L.ctm_workspace_bytes(2, D, chi, ctypes.byref(fixed))), D
    bad = B.default_opts(k_tracked=-2)
    assert L.ctm_workspace_bytes(2, 4, 64, ctypes.byref(bad)) == 0
    neg = B.default_opts(qr_reg_eps=-1.0)
    assert L.ctm_workspace_bytes(2, 4, 64, ctypes.byref(neg)) == 0


def test_kept_yz_adds_two_slots_per_tracked_step():
    # keeping Y and Z costs 2 max(k, 2) chi^2 D^4 doubles more, nothing else
    L = P.lib()
    for d, D, chi, k in [(2, 4, 64, 3), (2, 6, 144, 1), (2, 2, 16, 10)]:
        keep, rec = B.default_opts(k_tracked=k, grad_keep_yz=1), B.default_opts(k_tracked=k)
        extra = (L.ctm_workspace_bytes(d, D, chi, ctypes.byref(keep))
                 - L.ctm_workspace_bytes(d, D, chi, ctypes.byref(rec)))
        want = 2 * max(k, 2) * chi * chi * D**4 * 8
        assert want <= extra < want + 4096


def test_split_operand_planned_only_where_the_kernels_apply():
    L = P.lib()
    on, off = B.default_opts(edge_split=1), B.default_opts(edge_split=0)
    ws = lambda d, D, chi, o: L.ctm_workspace_bytes(d, D, chi, ctypes.byref(o))
    # d = 2, D <= 8: the prepared operand (and, for D <= 6, the reverse pass's
    # partial sums) are planned
    assert ws(2, 6, 144, on) > ws(2, 6, 144, off)
    assert ws(2, 8, 256, on) > ws(2, 8, 256, off)
    # other d, and chi^2 D^4 beyond 32-bit offsets: the double-layer product
    assert ws(3, 4, 64, on) == ws(3, 4, 64, off)
    assert ws(2, 8, 1024, on) == ws(2, 8, 1024, off)
    bad = B.default_opts(edge_split=2)
    assert L.ctm_workspace_bytes(2, 4, 64, ctypes.byref(bad)) == 0  # invalid options


def test_workspace_sizes_grow_with_problem():
    L = P.lib()
    small = L.ctm_workspace_bytes(2, 2, 16, None)
    mid = L.ctm_workspace_bytes(2, 4, 64, None)
    big = L.ctm_workspace_bytes(2, 6, 144, None)
    assert 0 < small < mid < big
    # Y and Z intermediates alone are chi^2 D^4 doubles each at D=6, chi=144
    assert big > 2 * 144 * 144 * 36 * 36 * 8
    assert L.ctm_workspace_bytes(0, 2, 16, None) == 0
    assert L.ctm_workspace_bytes_dl(2, 32, None) > 0
    assert L.ctm_qr_workspace_bytes(10, 20) == 0


def test_invalid_arguments_rejected_before_any_gpu_work():
    L = P.lib()
    ctx = ctypes.c_void_p()
    # null tensor
    rc = L.ctm_init(ctypes.byref(ctx), None, 2, 2, 16, None, None, 0, None)
    assert rc == B.CTM_EINVAL
    assert b"invalid" in L.ctm_last_error(None)
    # missing workspace (pointer value is never dereferenced on this path)
    fake = ctypes.c_void_p(0x1000)
    rc = L.ctm_init(ctypes.byref(ctx), fake, 2, 2, 16, None, None, 0, None)
    assert rc == B.CTM_EWORKSPACE
    # chi smaller than the bond dimension of the bulk tensor
    rc = L.ctm_init(ctypes.byref(ctx), fake, 2, 4, 8, None, fake, 1 << 40, None)
    assert rc == B.CTM_EINVAL
    # invalid precision
    o = B.default_opts()
    o.precision = 7
    rc = L.ctm_init(ctypes.byref(ctx), fake, 2, 2, 16, ctypes.byref(o), fake, 1 << 40, None)
    assert rc == B.CTM_EINVAL
    # null context on every context call
    assert L.ctm_step(None, 1, None) == B.CTM_EINVAL
    assert L.ctm_converge(None, 1e-10, 1, None, None) == B.CTM_EINVAL
    assert L.ctm_energy(None, None, None, 0.0, None) == B.CTM_EINVAL
    # QR shape check
    assert L.ctm_qr(fake, fake, fake, 4, 8, 0, fake, 1 << 20, None, None) == B.CTM_EINVAL
    assert L.ctm_qr(fake, fake, fake, 8, 4, 5, fake, 1 << 20, None, None) == B.CTM_EINVAL


def test_binding_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        P.Context(A=[[1.0]], chi=4)
