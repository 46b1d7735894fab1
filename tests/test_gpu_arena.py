"""The caller-owned arena, refactorization and input checks on the GPU.

* a factorization fits in the analysis bound, and a refactorization fits in exactly the
  bytes the first one used (same values, same sizes);
* an arena too small for the factor data stops the factorization with HSOLVE_ERR_OOM, and the
  plan then factors normally in a large enough one;
* solves with more right-hand sides than the arena holds at once run in batches and equal
  the one-batch solve column by column;
* GMRES after a refactorization repeats itself bitwise (its Krylov basis is re-carved);
* NaN / Inf in the values or the right-hand side give HSOLVE_ERR_INVALID;
* a non-SPD pivot is reported with and without the pivot overlap.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1611_03189_amd import problems as pb

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1611_03189_amd import hsolve as H  # noqa: E402


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_bound_fits_and_refactor_fits_in_used_bytes():
    say("arena bound / used")
    p = pb.lognormal(48, 2, 1.0, 31)
    S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=16, eps=1e-2)
    v = dev(p.values)
    r = dev(pb.rhs(p.n, 3, 5))
    big = torch.empty(S.arena_bound, dtype=torch.uint8, device="cuda")
    S.factor(v, arena=big)
    z1 = S.apply(r).cpu().numpy()
    used = S.stats()["device_bytes"]
    assert 0 < used <= S.arena_bound
    small = torch.empty(used, dtype=torch.uint8, device="cuda")
    S.factor(v, arena=small)
    z2 = S.apply(r).cpu().numpy()
    assert np.array_equal(z1, z2)
    S.factor(p.values)                     # host values, the plan's own arena
    assert np.array_equal(S.apply(r).cpu().numpy(), z1)
    S.close()


def test_too_small_arena_is_oom_then_recovers():
    say("arena oom")
    p = pb.poisson(24, 3)
    S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=64, eps=1e-2, max_nrhs=1)
    v = dev(p.values)
    S.factor(v)
    st = S.stats()
    used, fb = st["device_bytes"], st["factor_bytes"]
    z_ok = S.apply(dev(pb.rhs(p.n, 1, 3))).cpu().numpy()
    # the pattern and the transient regions fit, half of the factor data does not: the
    # factor region runs out part way through the levels
    tight = torch.empty(used - fb // 2, dtype=torch.uint8, device="cuda")
    with pytest.raises(H.HSolveError) as e:
        S.factor(v, arena=tight)
    assert e.value.status == -4
    with pytest.raises(H.HSolveError) as e:
        S.apply(dev(pb.rhs(p.n, 1, 3)))
    assert e.value.status == -6             # no factorization after the failure
    S.factor(v, arena=torch.empty(S.arena_bound, dtype=torch.uint8, device="cuda"))
    assert np.array_equal(S.apply(dev(pb.rhs(p.n, 1, 3))).cpu().numpy(), z_ok)
    S.close()


@pytest.mark.parametrize("krylov", ["pcg", "stationary"])
def test_solve_in_batches_equals_one_batch(krylov):
    say("batched columns", krylov)
    p = pb.lognormal(32, 2, 1.0, 8)
    B = dev(pb.rhs(p.n, 9, 12))
    S1 = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=16, eps=1e-2, krylov=krylov, max_nrhs=9)
    S1.factor(dev(p.values))
    X1, st1 = S1.solve(B)
    # an arena that holds the factor and the workspace of only a few columns
    S2 = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=16, eps=1e-2, krylov=krylov, max_nrhs=1)
    S2.factor(dev(p.values))
    used = S2.stats()["device_bytes"]
    S2.factor(dev(p.values), arena=torch.empty(used, dtype=torch.uint8, device="cuda"))
    X2, st2 = S2.solve(B)
    # one batch of nine runs the GEMM sweeps, batches of fewer than four the row/column
    # sweeps: the same solutions to the solver's accuracy, the same iteration counts
    assert st2["converged"] and abs(st1["iterations"] - st2["iterations"]) <= 1
    x1, x2 = X1.cpu().numpy(), X2.cpu().numpy()
    assert np.linalg.norm(x1 - x2) <= 1e-8 * np.linalg.norm(x1)
    Z1 = S1.apply(B).cpu().numpy()
    Z2 = S2.apply(B).cpu().numpy()
    assert np.linalg.norm(Z1 - Z2) <= 1e-13 * np.linalg.norm(Z1)
    S1.close()
    S2.close()


def test_gmres_after_refactor_is_bitwise_repeatable():
    say("gmres refactor")
    p = pb.lognormal(40, 2, 1.0, 21)
    b = dev(pb.rhs(p.n, 1, 4)[:, 0])
    v = dev(p.values)
    S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=16, eps=1e-2, krylov="gmres", restart=30)
    S.factor(v)
    x1, st1 = S.solve(b)
    S.factor(v)
    x2, st2 = S.solve(b)
    assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy()) and st1["iterations"] == st2["iterations"]
    F = O.factor(p.row_ptr, p.col_idx, p.values, p.coords, leaf=16, eps=1e-2, variant=O.GC)
    xr, itr, _ = O.gmres(p.to_scipy(), pb.rhs(p.n, 1, 4)[:, 0], lambda r: O.apply(F, r), restart=30)
    assert abs(st2["iterations"] - itr) <= 1
    S.close()


def test_non_finite_inputs_are_invalid():
    say("nan inputs")
    p = pb.poisson(12, 2)
    S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=8, eps=1e-2)
    bad = p.values.copy()
    bad[5] = np.nan
    with pytest.raises(H.HSolveError) as e:
        S.factor(dev(bad))
    assert e.value.status == -1
    bad[5] = np.inf
    with pytest.raises(H.HSolveError) as e:
        S.factor(bad)
    assert e.value.status == -1
    S.factor(dev(p.values))
    b = pb.rhs(p.n, 2, 1)
    b[3, 1] = np.nan
    with pytest.raises(H.HSolveError) as e:
        S.solve(dev(b))
    assert e.value.status == -1
    S.close()


@pytest.mark.parametrize("overlap", [True, False])
def test_not_spd_reported_with_and_without_overlap(overlap):
    say("not spd, overlap", overlap)
    p = pb.poisson(16, 2)
    vals = p.values.copy()
    diag = np.repeat(np.arange(p.n), np.diff(p.row_ptr)) == p.col_idx
    vals[diag] -= 8.0
    S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=4, eps=0.1, overlap_pivots=overlap)
    with pytest.raises(H.NotSPD):
        S.factor(dev(vals))
    st = S.stats()
    assert st["fail_level"] == S.depth - 1 and st["fail_node"] >= 0
    S.close()
