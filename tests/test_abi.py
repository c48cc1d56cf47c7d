"""The C ABI library loads, exports every declared symbol, and validates its
arguments on the host before any device work (CPU only)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1310_5954_amd import _lib as L
from paper_1310_5954_amd.api import Problem
from workload.configs import build_case

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "letkf.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(letkf_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    names = _declared()
    assert "letkf_create" in names and "letkf_submit_frame" in names
    for n in names:
        assert hasattr(lib, n), n


def _problem(**over):
    case = build_case(1)
    kw = dict(n_act=case.n_act, n_sub=case.n_sub, m=case.m, a1=case.a1, a2=case.a2, sigma_v=case.sigma_v,
              r_inv=case.r_inv, d_rowptr=case.D.rowptr, d_col=case.D.col, d_val=case.D.val,
              est_ptr=case.dmap.est_ptr, est_act=case.dmap.est_act, est_w=case.dmap.est_w,
              obs_ptr=case.dmap.obs_ptr, obs_sub=case.dmap.obs_sub, obs_taper=case.dmap.obs_taper)
    kw.update(over)
    return Problem(**kw)


def test_workspace_size_grows_with_precision_and_debug():
    pr = _problem()
    s64 = pr.workspace_size(L.FP64)
    s32 = pr.workspace_size(L.FP32)
    sdbg = pr.workspace_size(L.FP64, L.FLAG_DEBUG)
    assert 0 < s32 < s64 < sdbg
    assert s64 % 256 == 0


@pytest.mark.parametrize("over,needle", [
    (dict(m=1), "m must be"),
    (dict(m=257), "m must be"),
    (dict(n_act=0), "n_act"),
    (dict(sigma_v=-1.0), "sigma_v"),
    (dict(inflation=0.0), "inflation"),
])
def test_invalid_dims_and_model_rejected(over, needle):
    pr = _problem(**over)
    b = C.c_size_t()
    rc = L.lib().letkf_workspace_size(C.byref(pr.dims), C.byref(pr.model), C.byref(pr.map), L.FP64, 0, C.byref(b))
    assert rc == L.EINVAL
    assert needle in L.lib().letkf_last_error().decode()


def test_large_ensembles_fp64_only():
    """m in 129..256 is accepted in FP64 only (the multi-launch analysis), with
    scratch for two 256 x 256 FP64 matrices per domain, and without pistons.
    (At m = 128 the FP64 workspace holds one copy of A per domain, its lower
    triangle packed: 128 * 129 / 2 values.)"""
    b = C.c_size_t()
    pr128, pr200 = _problem(m=128), _problem(m=200)
    args = lambda pr: (C.byref(pr.dims), C.byref(pr.model), C.byref(pr.map))
    assert L.lib().letkf_workspace_size(*args(pr128), L.FP64, 0, C.byref(b)) == L.OK
    s128 = b.value
    assert L.lib().letkf_workspace_size(*args(pr200), L.FP64, 0, C.byref(b)) == L.OK
    n_dom = pr200.map.n_domains
    assert b.value - (s128 - n_dom * (128 * 129 // 2) * 8) >= n_dom * 2 * 256 * 256 * 8
    for prec in (L.FP32, L.BF16):
        assert L.lib().letkf_workspace_size(*args(pr200), prec, 0, C.byref(b)) == L.EINVAL
        assert "needs LETKF_FP64" in L.lib().letkf_last_error().decode()
    assert L.lib().letkf_workspace_size(*args(pr200), L.FP64, L.FLAG_PISTONS, C.byref(b)) == L.EINVAL
    assert "m <= 128" in L.lib().letkf_last_error().decode()


def test_invalid_map_rejected():
    case = build_case(1)
    w = case.dmap.est_w.copy()
    w[0] = 0.5                      # weights of actuator no longer sum to 1
    pr = _problem(est_w=w)
    b = C.c_size_t()
    assert L.lib().letkf_workspace_size(C.byref(pr.dims), C.byref(pr.model), C.byref(pr.map), L.FP64, 0,
                                        C.byref(b)) == L.EINVAL
    sub = case.dmap.obs_sub.copy()
    sub[3] = case.n_sub + 5         # out of range
    pr = _problem(obs_sub=sub)
    assert L.lib().letkf_workspace_size(C.byref(pr.dims), C.byref(pr.model), C.byref(pr.map), L.FP64, 0,
                                        C.byref(b)) == L.EINVAL
    col = case.D.col.copy()
    col[0] = -1
    pr = _problem(d_col=col)
    assert L.lib().letkf_workspace_size(C.byref(pr.dims), C.byref(pr.model), C.byref(pr.map), L.FP64, 0,
                                        C.byref(b)) == L.EINVAL


def test_bad_precision_and_flags_rejected():
    pr = _problem()
    b = C.c_size_t()
    assert L.lib().letkf_workspace_size(C.byref(pr.dims), C.byref(pr.model), C.byref(pr.map), 7, 0,
                                        C.byref(b)) == L.EINVAL
    assert L.lib().letkf_workspace_size(C.byref(pr.dims), C.byref(pr.model), C.byref(pr.map), 0, 0x80,
                                        C.byref(b)) == L.EINVAL


def test_create_rejects_small_workspace_before_device_work():
    pr = _problem()
    h = C.c_void_p()
    X0 = np.zeros((pr.n, pr.m))
    rc = L.lib().letkf_create(C.byref(pr.dims), C.byref(pr.model), C.byref(pr.map), L.FP64, 0,
                              X0.ctypes.data_as(C.POINTER(C.c_double)), C.c_void_p(256), 1024, None, C.byref(h))
    assert rc == L.ENOMEM and not h.value
    # the message reports the size letkf_workspace_size gives (computed before
    # the half-built handle is released)
    assert f"need {pr.workspace_size(L.FP64)} bytes" in L.lib().letkf_last_error().decode()
    X0[0, 0] = np.nan
    rc = L.lib().letkf_create(C.byref(pr.dims), C.byref(pr.model), C.byref(pr.map), L.FP64, 0,
                              X0.ctypes.data_as(C.POINTER(C.c_double)), C.c_void_p(256), 1 << 40, None, C.byref(h))
    assert rc == L.ENUMERIC


def test_strerror_covers_codes():
    for code in (L.OK, L.EINVAL, L.ENOMEM, L.EAGAIN, L.EDEVICE, L.ENUMERIC, L.ESTATE):
        assert L.lib().letkf_strerror(code)


def test_server_reserved_bytes_is_a_host_query():
    """The server's own share of an arena is known before any device work
    (it sizes HBM budgets); 256-byte aligned like every arena region."""
    n = L.lib().letkf_server_reserved_bytes()
    assert n > 0 and n % 256 == 0


def test_fp32_rotations_flag_needs_bf16():
    """LETKF_FLAG_FP32_ROTATIONS (the opt-in FP32 Jacobi rotations) is a
    variant of the BF16 path only."""
    pr = _problem()
    b = C.c_size_t()
    args = (C.byref(pr.dims), C.byref(pr.model), C.byref(pr.map))
    assert L.lib().letkf_workspace_size(*args, L.BF16, L.FLAG_FP32_ROTATIONS, C.byref(b)) == L.OK
    for prec in (L.FP64, L.FP32):
        assert L.lib().letkf_workspace_size(*args, prec, L.FLAG_FP32_ROTATIONS, C.byref(b)) == L.EINVAL
        assert "needs LETKF_BF16" in L.lib().letkf_last_error().decode()


def test_obs_instant_values():
    """obs_instant 0 (H = [D 0]) and 1 (H = [0 D]) are accepted, nothing else."""
    b = C.c_size_t()
    for v, rc in ((0, L.OK), (1, L.OK), (2, L.EINVAL), (-1, L.EINVAL)):
        pr = _problem(obs_instant=v)
        assert L.lib().letkf_workspace_size(C.byref(pr.dims), C.byref(pr.model), C.byref(pr.map), L.FP64, 0,
                                            C.byref(b)) == rc, v
    assert "obs_instant" in L.lib().letkf_last_error().decode()


def test_server_refuses_instances_larger_than_its_staging():
    """A batch stages each frame's slopes and means in slots of 2^18 values, so
    an instance with p or n_act above that could never be batched: the server
    refuses it (arguments are checked before the server handle is used, so a
    null server shows it without a GPU).  A problem within the limit gets to
    the null-server check."""
    n_sub = (1 << 17) + 1                      # p = 2^18 + 2 slopes
    p = 2 * n_sub
    pr = Problem(n_act=4, n_sub=n_sub, m=4, a1=np.ones(4), a2=np.zeros(4), sigma_v=0.0, r_inv=np.ones(p),
                 d_rowptr=np.zeros(p + 1, np.int32), d_col=np.zeros(0, np.int32), d_val=np.zeros(0),
                 est_ptr=[0, 4], est_act=[0, 1, 2, 3], est_w=np.ones(4), obs_ptr=[0, 0],
                 obs_sub=np.zeros(0, np.int32), obs_taper=np.zeros(0))
    X0 = np.zeros((pr.n, pr.m))
    h = C.c_void_p()
    rc = L.lib().letkf_server_add(None, C.byref(pr.dims), C.byref(pr.model), C.byref(pr.map), L.FP64, 0,
                                  X0.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h))
    assert rc == L.EINVAL and not h.value
    assert "staging" in L.lib().letkf_last_error().decode()
    small = _problem()
    X0 = np.zeros((small.n, small.m))
    rc = L.lib().letkf_server_add(None, C.byref(small.dims), C.byref(small.model), C.byref(small.map), L.FP64, 0,
                                  X0.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h))
    assert rc == L.EINVAL and "null server" in L.lib().letkf_last_error().decode()
