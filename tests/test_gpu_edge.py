"""Degenerate and boundary inputs through the C ABI on the GPU: one unknown, a right-hand
side of zeros, a block with a zero column beside a nonzero one, a three-unknown chain, and
leaf pairs of exactly the largest super node the kernels take (512)."""
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

TOL = 1e-10


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_single_unknown():
    say("n1")
    p = pb.poisson(1, 1)                     # A = [2]
    assert p.n == 1
    S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=16, eps=1e-2)
    S.factor(dev(p.values))
    z = S.apply(dev(np.array([3.0]))).cpu().numpy()
    assert abs(z[0] - 1.5) <= 1e-15
    x, st = S.solve(dev(np.array([-4.0])))
    assert abs(x.cpu().numpy()[0] + 2.0) <= 1e-15 and st["converged"] and st["iterations"] <= 1
    S.close()


@pytest.mark.parametrize("krylov", ["pcg", "fpcg", "gmres"])
def test_zero_rhs(krylov):
    say("zero rhs", krylov)
    p = pb.poisson(16, 2)
    S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=8, eps=1e-2, krylov=krylov)
    S.factor(dev(p.values))
    x, st = S.solve(dev(np.zeros(p.n)))
    assert np.all(x.cpu().numpy() == 0.0) and st["converged"] and st["iterations"] == 0
    S.close()


def test_zero_column_beside_nonzero():
    say("zero column in a block")
    p = pb.poisson(24, 2)
    b = pb.rhs(p.n, 2, 41)
    b[:, 0] = 0.0
    S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=8, eps=1e-2)
    S.factor(dev(p.values))
    X, st = S.solve(dev(b))
    X = X.cpu().numpy()
    x1, _ = S.solve(dev(b[:, 1]))
    assert np.all(X[:, 0] == 0.0)
    assert np.array_equal(X[:, 1], x1.cpu().numpy())
    A = p.to_scipy()
    assert np.linalg.norm(b[:, 1] - A @ X[:, 1]) / np.linalg.norm(b[:, 1]) <= 2 * TOL
    S.close()


def test_three_unknown_chain_matches_oracle():
    say("chain n3")
    p = pb.chain(3)
    F = O.factor(p.row_ptr, p.col_idx, p.values, p.coords, leaf=1, eps=1e-2, variant=O.GC)
    S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=1, eps=1e-2)
    S.factor(dev(p.values))
    r = pb.rhs(p.n, 2, 43)
    z = S.apply(dev(r)).cpu().numpy()
    z_ref = O.apply(F, r)
    assert np.linalg.norm(z - z_ref) / np.linalg.norm(z_ref) <= TOL
    S.close()


def test_largest_leaf_pairs():
    """16^3 Poisson with leaves of 256: the first super nodes have 512 unknowns, the largest
    the compression and pivot kernels take; the apply matches the oracle."""
    say("leaf pairs of 512")
    p = pb.poisson(16, 3)
    F = O.factor(p.row_ptr, p.col_idx, p.values, p.coords, leaf=256, eps=1e-2, variant=O.GC)
    S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=256, eps=1e-2)
    S.factor(dev(p.values))
    for d in F.levels:
        assert S.ranks(d).tolist() == F.ranks(d), d
    r = pb.rhs(p.n, 1, 45)
    z = S.apply(dev(r)).cpu().numpy()
    z_ref = O.apply(F, r)
    assert np.linalg.norm(z - z_ref) / np.linalg.norm(z_ref) <= TOL
    S.close()


def test_largest_leaf_pairs_gc_four_vectors():
    """The same 512-unknown leaf pairs with GC keeping four vectors (1, x, y, z): Z =
    [phi_s, A_sw phi_w] has 8 columns, so up to 8 GC reflectors are applied as one block,
    whose LDS buffers (3 x 8 x 512 doubles) are the largest the global-matrix compression
    holds. Ranks equal and the apply within the FP64 bar of the oracle."""
    say("leaf pairs of 512, GC with 4 vectors")
    p = pb.poisson(16, 3)
    c = p.coords
    x = (c - c.mean(0)) / np.ptp(c, 0)
    phi = np.asfortranarray(np.column_stack([np.ones(p.n), x[:, 0], x[:, 1], x[:, 2]]))
    F = O.factor(p.row_ptr, p.col_idx, p.values, p.coords, leaf=256, eps=1e-2, variant=O.GC, phi=phi)
    S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=256, eps=1e-2, phi=phi)
    S.factor(dev(p.values))
    assert F.tie_margin > 1e-9
    for d in F.levels:
        assert S.ranks(d).tolist() == F.ranks(d), d
    r = pb.rhs(p.n, 1, 46)
    z = S.apply(dev(r)).cpu().numpy()
    z_ref = O.apply(F, r)
    assert np.linalg.norm(z - z_ref) / np.linalg.norm(z_ref) <= TOL
    assert np.max(np.abs(z - z_ref)) / np.max(np.abs(z_ref)) <= TOL
    # each kept vector is preserved exactly: A_H^{-1} A phi_j = phi_j (the GC invariant)
    for j in range(phi.shape[1]):
        zj = S.apply(dev(p.dense() @ phi[:, j])).cpu().numpy()
        assert np.max(np.abs(zj - phi[:, j])) / np.max(np.abs(phi[:, j])) < 1e-10, j
    S.close()
