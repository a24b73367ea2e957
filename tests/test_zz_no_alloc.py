"""The no-allocation entry point sp2_run_dense_noalloc, called through the C
ABI: its result equals, bit for bit, that of the context entry points
(sp2_create, sp2_init_dense, sp2_run, sp2_get_density, sp2_get_info,
sp2_get_history) on the same input with the same options, on two calls in a
row (the second with a smaller input, so the scratch holds the first call's
contents), in every precision; it matches the FP64 oracle within the
precision's Frobenius tolerance; inputs larger than its scratch and options
it does not support are rejected before any work is queued."""
import ctypes
import math

import numpy as np
import pytest

import oracle
from workloads import dense_instance
from tests.gpu_helpers import print_case

pytestmark = pytest.mark.gpu

D_TOL = {"fp64": 1e-11, "fp32": 2e-5, "bf16x3": 2e-4}
CAP = 202


def _lib():
    import paper_1507_02087_amd as sp2
    return sp2, sp2.load_library()


def _opts(sp2, prec, **kw):
    opt = sp2.Options()
    sp2.load_library().sp2_default_options(ctypes.byref(opt))
    opt.precision = sp2.PRECISIONS[prec]
    opt.tail_split = 1
    for k, v in kw.items():
        setattr(opt, k, v)
    return opt


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _context_run(sp2, lib, F, inst, opt):
    import torch
    n = F.shape[0]
    h = ctypes.c_void_p()
    assert lib.sp2_create(ctypes.byref(h), 0, _stream()) == sp2.OK
    try:
        st = lib.sp2_init_dense(h, ctypes.c_void_p(F.data_ptr()), n, F.stride(0),
                                inst.lambda_min, inst.lambda_max, inst.n_occ,
                                ctypes.byref(opt))
        assert st == sp2.OK, lib.sp2_last_error(h)
        st = lib.sp2_run(h)
        D = torch.empty((n, n), dtype=torch.float64, device="cuda")
        assert lib.sp2_get_density(h, ctypes.c_void_p(D.data_ptr()), n, 1) == sp2.OK
        it, sq, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        assert lib.sp2_get_info(h, ctypes.byref(it), ctypes.byref(sq),
                                ctypes.byref(ms)) == sp2.OK
        v = np.full(CAP, np.nan)
        ln = ctypes.c_int32()
        assert lib.sp2_get_history(h, CAP, ctypes.byref(ln), ctypes.c_void_p(v.ctypes.data),
                                   None, None, None, None) == sp2.OK
        return st, D, it.value, sq.value, v
    finally:
        lib.sp2_destroy(h)


def _noalloc_run(sp2, lib, F, inst, opt, ldd=None):
    import torch
    n = F.shape[0]
    ldd = ldd or n
    D = torch.full((n, ldd), -7.0, dtype=torch.float64, device="cuda")
    v = np.full(CAP, -1.0)
    it, sq = ctypes.c_int32(-1), ctypes.c_int32(-1)
    st = lib.sp2_run_dense_noalloc(0, _stream(), ctypes.c_void_p(F.data_ptr()), n,
                                   F.stride(0), inst.lambda_min, inst.lambda_max,
                                   inst.n_occ, ctypes.byref(opt),
                                   ctypes.c_void_p(D.data_ptr()), ldd, 1, CAP,
                                   ctypes.c_void_p(v.ctypes.data), ctypes.byref(it),
                                   ctypes.byref(sq))
    torch.cuda.synchronize()
    return st, D[:, :n], it.value, sq.value, v


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_noalloc_equals_context_run_twice(prec):
    import torch
    sp2, lib = _lib()
    for n, gap, seed in ((700, 0.1, 71), (300, 0.05, 72)):
        inst = dense_instance(n, n // 2, -1.0, 1.0, gap, seed=seed)
        F = torch.from_numpy(inst.F).to("cuda:0")
        print_case(f"no-alloc n={n} prec={prec}")
        opt = _opts(sp2, prec)
        a = _context_run(sp2, lib, F, inst, opt)
        b = _noalloc_run(sp2, lib, F, inst, opt)
        assert a[0] == sp2.OK and b[0] == sp2.OK, (a[0], b[0])
        assert (b[2], b[3]) == (a[2], a[3])
        assert torch.equal(a[1], b[1])
        sq = a[3]
        assert np.array_equal(a[4][:sq], b[4][:sq]) and np.all(np.isnan(b[4][sq:]))
        ref = oracle.sp2(inst.F, inst.lambda_min, inst.lambda_max, inst.n_occ)
        err = float(np.linalg.norm(b[1].cpu().numpy() - ref.X)) / math.sqrt(inst.n_occ)
        print(f"  n_iter={b[2]} squares={b[3]} err vs oracle {err:.2e}", flush=True)
        assert err < D_TOL[prec]


def test_noalloc_leading_dimension_and_trivial_cases():
    import torch
    sp2, lib = _lib()
    inst = dense_instance(130, 65, -1.0, 1.0, 0.1, seed=73)
    F = torch.from_numpy(inst.F).to("cuda:0")
    opt = _opts(sp2, "fp32")
    a = _context_run(sp2, lib, F, inst, opt)
    b = _noalloc_run(sp2, lib, F, inst, opt, ldd=160)
    assert b[0] == sp2.OK and torch.equal(a[1], b[1])
    for n_occ, want in ((0, 0.0), (130, 1.0)):
        inst.n_occ = n_occ
        st, D, it, sq, v = _noalloc_run(sp2, lib, F, inst, opt)
        assert st == sp2.OK and it == 0 and sq == 0 and np.all(np.isnan(v))
        assert torch.equal(D.cpu(), want * torch.eye(130, dtype=torch.float64))


def test_noalloc_rejects_oversized_input_and_unsupported_options():
    import torch
    sp2, lib = _lib()
    inst = dense_instance(64, 32, -1.0, 1.0, 0.1, seed=74)
    F = torch.from_numpy(inst.F).to("cuda:0")
    for kw in (dict(norm=sp2.NORMS["mixed"]), dict(norm=sp2.NORMS["spectral"]),
               dict(tail_split=4), dict(kernel_timing=1)):
        st, D, it, sq, v = _noalloc_run(sp2, lib, F, inst, _opts(sp2, "fp64", **kw))
        assert st == sp2.INVALID_ARG, kw
        assert it == -1 and float(D.max()) == -7.0   # nothing was run
    big = torch.zeros((3000, 3000), dtype=torch.float64, device="cuda")
    big.fill_diagonal_(0.5)
    inst_big = dense_instance(64, 32, -1.0, 1.0, 0.1, seed=75)
    inst_big.n_occ = 1500
    for prec in ("fp64", "fp32", "bf16x3"):
        st, D, it, sq, v = _noalloc_run(sp2, lib, big, inst_big, _opts(sp2, prec))
        assert st == sp2.INVALID_ARG, prec
        assert it == -1
