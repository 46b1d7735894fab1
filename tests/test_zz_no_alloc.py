"""hsolve_apply_static (the apply for callers that cannot allocate) against hsolve_apply,
through the C ABI: bitwise equal results on two calls in a row, the second with a smaller
input (fewer right-hand sides, then a smaller plan), in FP64 and with the FP32 solve phase;
a call whose solve vectors exceed the static scratch is refused with HSOLVE_ERR_OOM."""
import ctypes
import sys

import numpy as np
import pytest

from paper_1611_03189_amd import problems as pb

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1611_03189_amd import hsolve as H  # noqa: E402


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def _static(S, R):
    """hsolve_apply_static on the (nrhs, n) row-major tensor R (= n x nrhs column-major)."""
    Z = torch.empty_like(R)
    st = S._lib.hsolve_apply_static(S._h, R.shape[0], ctypes.c_void_p(R.data_ptr()), S.n,
                                    ctypes.c_void_p(Z.data_ptr()), S.n)
    return st, Z


def _arena(S, R):
    Z = torch.empty_like(R)
    st = S._lib.hsolve_apply(S._h, R.shape[0], ctypes.c_void_p(R.data_ptr()), S.n,
                             ctypes.c_void_p(Z.data_ptr()), S.n)
    return st, Z


@pytest.mark.parametrize("apply_prec", [64, 32])
def test_static_apply_equals_apply_twice_then_smaller(apply_prec):
    say("apply_static", apply_prec)
    big = pb.lognormal(40, 2, 1.0, 13)
    small = pb.poisson(12, 2)
    S1 = H.HSolver(big.row_ptr, big.col_idx, coords=big.coords, leaf=16, eps=1e-2, apply_prec=apply_prec)
    S1.factor(torch.from_numpy(big.values).cuda())
    S2 = H.HSolver(small.row_ptr, small.col_idx, coords=small.coords, leaf=8, eps=1e-2, apply_prec=apply_prec)
    S2.factor(torch.from_numpy(small.values).cuda())
    # six columns first: the sweeps run as grouped GEMMs on the static vectors
    calls = [(S1, 6, 40), (S1, 3, 41), (S1, 1, 42), (S2, 2, 43), (S2, 1, 44)]
    for S, nrhs, seed in calls:
        R = torch.from_numpy(np.ascontiguousarray(pb.rhs(S.n, nrhs, seed).T)).cuda()
        st_s, Zs = _static(S, R)
        st_a, Za = _arena(S, R)
        assert st_s == 0 and st_a == 0, (st_s, st_a)
        assert torch.equal(Zs, Za), (S.n, nrhs)
        assert torch.isfinite(Zs).all()
    # the binding's method goes through the same entry point
    r = torch.from_numpy(pb.rhs(S1.n, 1, 45)[:, 0]).cuda()
    assert torch.equal(S1.apply_static(r), S1.apply(r))
    S1.close()
    S2.close()


def test_static_apply_rejects_more_than_the_scratch_holds():
    say("apply_static too large")
    p = pb.poisson(64, 2)
    S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=16, eps=1e-2)
    S.factor(torch.from_numpy(p.values).cuda())
    vlen = p.n + sum(int(S.ranks(d).sum()) for d in range(S.depth))
    nrhs = (64 << 20) // (2 * 8 * vlen) + 8               # beyond the 64 MiB scratch
    R = torch.zeros(nrhs, p.n, dtype=torch.float64, device="cuda")
    st, _ = _static(S, R)
    assert st == -4
    assert b"static scratch" in S._lib.hsolve_last_error(S._h)
    # a call that fits still works after the refusal
    R1 = torch.from_numpy(np.ascontiguousarray(pb.rhs(p.n, 2, 3).T)).cuda()
    st1, Z1 = _static(S, R1)
    st2, Z2 = _arena(S, R1)
    assert st1 == 0 and st2 == 0 and torch.equal(Z1, Z2)
    S.close()
