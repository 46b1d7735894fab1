"""GPU (HIP, gfx950) path vs the FP64 CPU oracle, through the C ABI.

Bar (FP64 path): rank vectors equal level by level, and ||z_gpu - z_oracle|| /
||z_oracle|| <= 1e-10 for z = A_H^{-1} r on the same seeded r. Properties that hold at any
size are checked at the full workload sizes (GC invariant A_H^{-1} A 1 = 1, PCG reaching
1e-10 true residual). Each case prints its name before touching the GPU.
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

TOL = 1e-10


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def run_pair(p, leaf, eps, variant, nrhs=2, seed=7, phi=None, coords="grid", F=None, **kw):
    c = p.coords if coords == "grid" else None
    if F is None:
        F = O.factor(p.row_ptr, p.col_idx, p.values, c, leaf=leaf, eps=eps,
                     variant=O.GC if variant == "gc" else O.LORASP, phi=phi,
                     eps_schedule=kw.get("eps_schedule", "constant"))
    S = H.HSolver(p.row_ptr, p.col_idx, coords=c, leaf=leaf, eps=eps, variant=variant, phi=phi, **kw)
    S.factor(torch.from_numpy(p.values).cuda())
    r = pb.rhs(p.n, nrhs, seed)
    z_ref = O.apply(F, r)
    z = S.apply(torch.from_numpy(np.ascontiguousarray(r)).cuda()).cpu().numpy()
    return F, S, r, z_ref, z


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def max_rel(a, b):
    """Largest entry error relative to the largest entry: the max-norm companion of rel()."""
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def check_parity(F, S, z, z_ref, name, tol=TOL):
    """The FP64 bar: equal rank vectors (only where no rank decision sat within 1e-9 of the
    threshold, reading R16), and z within tol of the oracle in the 2-norm and the max-norm."""
    say(name, f"tie margin {F.tie_margin:.2e} rel {rel(z, z_ref):.2e} max_rel {max_rel(z, z_ref):.2e}")
    assert F.tie_margin > 1e-9, (name, "rank decision too close to the threshold; change the case")
    for d in F.levels:
        assert S.ranks(d).tolist() == F.ranks(d), (name, d)
    assert rel(z, z_ref) <= tol, (name, rel(z, z_ref))
    assert max_rel(z, z_ref) <= tol, (name, max_rel(z, z_ref))


PARITY = [
    ("c1_poisson2d_32_leaf16_gc", lambda: pb.poisson(32, 2), 16, 1e-2, "gc"),
    ("c1_poisson2d_32_leaf16_lorasp", lambda: pb.poisson(32, 2), 16, 1e-2, "lorasp"),
    ("poisson2d_30_ragged_leaf8_gc", lambda: pb.poisson(30, 2), 8, 0.05, "gc"),
    ("lognormal2d_48_s2_leaf8_gc", lambda: pb.lognormal(48, 2, 2.0, 1002), 8, 1e-2, "gc"),
    ("poisson3d_12_leaf16_gc", lambda: pb.poisson(12, 3), 16, 1e-2, "gc"),
    ("poisson3d_16_leaf64_gc", lambda: pb.poisson(16, 3), 64, 1e-2, "gc"),
    ("poisson3d_16_leaf64_eps1e-4", lambda: pb.poisson(16, 3), 64, 1e-4, "gc"),
    ("poisson3d_8_leaf8_lorasp", lambda: pb.poisson(8, 3), 8, 0.1, "lorasp"),
    ("chain_300_leaf6_gc", lambda: pb.chain(300), 6, 0.1, "gc"),
    ("single_leaf_n20", lambda: pb.poisson(20, 1), 64, 1e-2, "gc"),
]


@pytest.mark.parametrize("name,make,leaf,eps,variant", PARITY, ids=[c[0] for c in PARITY])
def test_apply_matches_oracle(name, make, leaf, eps, variant):
    say(name)
    p = make()
    F, S, r, z_ref, z = run_pair(p, leaf, eps, variant)
    check_parity(F, S, z, z_ref, name)
    S.close()


def poly_phi(p, k):
    """k smooth vectors on the grid coordinates (1, x, y, xy, x^2), columns of an n x k array."""
    c = p.coords
    x = (c - c.mean(0)) / np.ptp(c, 0)
    cols = [np.ones(p.n), x[:, 0], x[:, 1], x[:, 0] * x[:, 1], x[:, 0] ** 2]
    return np.asfortranarray(np.column_stack(cols[:k]))


WIDE = [("gc_1vec", "gc", 1), ("gc_3vec", "gc", 3), ("gc_5vec", "gc", 5), ("lorasp", "lorasp", 0)]


@pytest.mark.parametrize("name,variant,k", WIDE, ids=[c[0] for c in WIDE])
def test_wide_super_nodes_match_oracle(name, variant, k):
    """Leaves of 256 unknowns (2-D Poisson 64^2): the leaf compressions take the global-memory
    form of the reduction (more than 128 unknowns per super node). With GC the kept vectors
    enter as a bordered tridiagonal (1 vector: 2 columns of Z = [phi_s, A_sw phi_w]), as one
    block reflector (3 vectors: 6 columns) and reflector by reflector (5 vectors: 10 columns)."""
    say("wide", name)
    p = pb.poisson(64, 2)
    phi = poly_phi(p, k) if k > 1 else None
    F, S, r, z_ref, z = run_pair(p, 256, 1e-2, variant, phi=phi)
    check_parity(F, S, z, z_ref, name)
    S.close()


@pytest.mark.parametrize("variant", ["gc", "lorasp"])
def test_eps_zero_exact_on_gpu(variant):
    say("eps0", variant)
    p = pb.poisson(16, 2)
    S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=8, eps=0.0, variant=variant)
    S.factor(torch.from_numpy(p.values).cuda())
    b = pb.rhs(p.n, 1, 5)[:, 0]
    x = np.linalg.solve(p.dense(), b)
    z = S.apply(torch.from_numpy(b).cuda()).cpu().numpy()
    # eps = 0 keeps every direction, so A_H = A (the extension lemma of section 5); the
    # apply equals the dense solve up to rounding, bounded here by 1e-12 kappa(A)
    assert rel(z, x) < 1e-12 * np.linalg.cond(p.dense())
    S.close()


def test_gc_eigenvector_phi_on_gpu():
    say("gc_eigenvector_p2")
    N = 24
    p = pb.poisson(N, 2)
    lam, V = np.linalg.eigh(p.dense())
    phi = np.asfortranarray(V[:, :2])
    F, S, r, z_ref, z = run_pair(p, 8, 0.2, "gc", phi=phi)
    assert rel(z, z_ref) <= TOL
    for j in range(2):
        zj = S.apply(torch.from_numpy(p.dense() @ phi[:, j]).cuda()).cpu().numpy()
        assert np.max(np.abs(zj - phi[:, j])) < 1e-10
    S.close()


def test_gc_three_vectors_on_gpu():
    # three preserved vectors: up to six kept basis columns per node
    say("gc_eigenvector_p3")
    N = 24
    p = pb.poisson(N, 2)
    lam, V = np.linalg.eigh(p.dense())
    phi = np.asfortranarray(V[:, :3])
    F, S, r, z_ref, z = run_pair(p, 8, 0.1, "gc", phi=phi)
    assert rel(z, z_ref) <= TOL
    for j in range(3):
        zj = S.apply(torch.from_numpy(p.dense() @ phi[:, j]).cuda()).cpu().numpy()
        assert np.max(np.abs(zj - phi[:, j])) < 1e-10
    S.close()


def test_multiple_rhs_equal_single():
    """Up to three right-hand sides run the row/column sweep kernels, every column in the
    order of the single-column sweep: bitwise equal to solving it alone."""
    say("multi_rhs")
    p = pb.poisson(32, 2)
    S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=16, eps=1e-2)
    S.factor(torch.from_numpy(p.values).cuda())
    B = pb.rhs(p.n, 3, 9)
    Z = S.apply(torch.from_numpy(np.ascontiguousarray(B)).cuda()).cpu().numpy()
    for j in range(3):
        zj = S.apply(torch.from_numpy(B[:, j].copy()).cuda()).cpu().numpy()
        assert np.array_equal(zj, Z[:, j])
    S.close()


@pytest.mark.parametrize("nrhs", [4, 8, 40])
def test_gemm_sweeps_for_many_rhs(nrhs):
    """Four or more right-hand sides run the sweeps as grouped GEMMs (40: two launches of 32
    and 8 columns per colour sweep). Each column matches the oracle to the FP64 bar and the
    single-column sweep to rounding, and does not depend on the other columns' values
    (bitwise)."""
    say("gemm sweeps", nrhs)
    p = pb.lognormal(32, 2, 1.0, 13)
    F = O.factor(p.row_ptr, p.col_idx, p.values, p.coords, leaf=16, eps=1e-2, variant=O.GC)
    S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=16, eps=1e-2)
    S.factor(torch.from_numpy(p.values).cuda())
    B = pb.rhs(p.n, nrhs, 19)
    Z = S.apply(torch.from_numpy(np.ascontiguousarray(B)).cuda()).cpu().numpy()
    Z_ref = O.apply(F, B)
    assert rel(Z, Z_ref) <= TOL and max_rel(Z, Z_ref) <= TOL
    for j in (0, nrhs - 1):
        zj = S.apply(torch.from_numpy(B[:, j].copy()).cuda()).cpu().numpy()
        assert rel(Z[:, j], zj) <= 1e-13
    B2 = B.copy()
    B2[:, 1:] = pb.rhs(p.n, nrhs - 1, 23)
    Z2 = S.apply(torch.from_numpy(np.ascontiguousarray(B2)).cuda()).cpu().numpy()
    assert np.array_equal(Z2[:, 0], Z[:, 0])
    S.close()


def test_batched_pcg_equals_single_columns():
    # all columns advance together with their own scalars; each must equal its own solve
    say("batched_pcg")
    p = pb.lognormal(40, 2, 1.0, 5)
    S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=16, eps=1e-2, tol=1e-10)
    S.factor(torch.from_numpy(p.values).cuda())
    # three columns: the row/column sweeps, bitwise equal to each column's own solve
    B = pb.rhs(p.n, 3, 11)
    B[:, 1] = 0.0
    X, st = S.solve(torch.from_numpy(np.ascontiguousarray(B)).cuda())
    X = X.cpu().numpy()
    A = p.to_scipy()
    most = 0
    for j in range(3):
        xj, stj = S.solve(torch.from_numpy(B[:, j].copy()).cuda())
        assert np.array_equal(xj.cpu().numpy(), X[:, j])
        most = max(most, stj["iterations"])
        if j == 1:
            assert np.all(X[:, 1] == 0.0) and stj["iterations"] == 0
        else:
            assert np.linalg.norm(B[:, j] - A @ X[:, j]) <= 2e-10 * np.linalg.norm(B[:, j])
    assert st["iterations"] == most and st["converged"]
    # six columns (the GEMM sweeps), one of them zero: each converges, the zero one stays zero,
    # and each agrees with its own single-column solve to the solver's accuracy
    B = pb.rhs(p.n, 6, 12)
    B[:, 4] = 0.0
    X, st = S.solve(torch.from_numpy(np.ascontiguousarray(B)).cuda())
    X = X.cpu().numpy()
    assert st["converged"] and np.all(X[:, 4] == 0.0)
    for j in (0, 5):
        xj, stj = S.solve(torch.from_numpy(B[:, j].copy()).cuda())
        assert np.linalg.norm(B[:, j] - A @ X[:, j]) <= 2e-10 * np.linalg.norm(B[:, j])
        assert rel(X[:, j], xj.cpu().numpy()) <= 1e-8
    S.close()


def test_refactor_and_run_twice_bitwise():
    say("determinism")
    p = pb.lognormal(32, 2, 1.0, 77)
    S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=8, eps=1e-2)
    v = torch.from_numpy(p.values).cuda()
    r = torch.from_numpy(pb.rhs(p.n, 1, 3)[:, 0]).cuda()
    S.factor(v)
    z1 = S.apply(r).cpu().numpy()
    S.factor(v)
    z2 = S.apply(r).cpu().numpy()
    assert np.array_equal(z1, z2)
    S.close()


@pytest.mark.parametrize("name,make,leaf,eps", [
    ("c1_poisson2d_32", lambda: pb.poisson(32, 2), 16, 1e-2),
    ("lognormal2d_64_s2", lambda: pb.lognormal(64, 2, 2.0, 1002), 16, 1e-2),
    ("poisson3d_16_leaf64", lambda: pb.poisson(16, 3), 64, 1e-2),
])
def test_pcg_matches_oracle(name, make, leaf, eps):
    say("pcg", name)
    p = make()
    A = p.to_scipy()
    b = pb.rhs(p.n, 1, 2001)[:, 0]
    F = O.factor(p.row_ptr, p.col_idx, p.values, p.coords, leaf=leaf, eps=eps, variant=O.GC)
    x_ref, it_ref, rel_ref = O.pcg(A, b, lambda r: O.apply(F, r), tol=TOL)
    S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=leaf, eps=eps)
    S.factor(torch.from_numpy(p.values).cuda())
    x, st = S.solve(torch.from_numpy(b).cuda())
    x = x.cpu().numpy()
    true_rel = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert st["converged"] and true_rel <= 2 * TOL, (true_rel, st)
    assert abs(st["iterations"] - it_ref) <= 1, (st["iterations"], it_ref)
    assert rel(x, x_ref) < 1e-8
    S.close()


def test_not_spd_is_reported():
    say("not_spd")
    p = pb.poisson(8, 2)
    vals = p.values.copy()
    diag = np.repeat(np.arange(p.n), np.diff(p.row_ptr)) == p.col_idx
    vals[diag] -= 8.0
    S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=4, eps=0.1)
    with pytest.raises(H.NotSPD):
        S.factor(torch.from_numpy(vals).cuda())
    st = S.stats()
    assert st["fail_level"] >= 0 and st["fail_node"] >= 0
    S.close()


@pytest.mark.slow
def test_c3_full_size_properties():
    """64^3 Poisson, leaf 64, eps 1e-2, GC: invariant and PCG at the benchmarked size."""
    say("c3_full_size")
    p, w = pb.workload("c3_poisson3d_64")
    S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=w["leaf"], eps=w["eps"])
    S.factor(torch.from_numpy(p.values).cuda())
    A = p.to_scipy()
    one = np.ones(p.n)
    z = S.apply(torch.from_numpy(A @ one).cuda()).cpu().numpy()
    assert np.max(np.abs(z - 1.0)) < 1e-9
    b = pb.rhs(p.n, 1, 2003)[:, 0]
    x, st = S.solve(torch.from_numpy(b).cuda())
    true_rel = np.linalg.norm(b - A @ x.cpu().numpy()) / np.linalg.norm(b)
    assert true_rel <= 2 * TOL and st["iterations"] <= 10, (true_rel, st)
    S.close()


def test_pivot_overlap_does_not_change_results():
    """The pivot blocks factored on the plan's second stream (default) or in order on its
    stream run the same kernels on the same data: bitwise equal applies."""
    say("pivot overlap on/off")
    p = pb.poisson(20, 3)
    r = torch.from_numpy(pb.rhs(p.n, 2, 47)).cuda()
    out = []
    for ov in (True, False):
        S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=64, eps=1e-2, overlap_pivots=ov)
        S.factor(torch.from_numpy(p.values).cuda())
        out.append(S.apply(r).cpu().numpy())
        S.close()
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("order", ["waiting", "index"])
@pytest.mark.parametrize("name,make,leaf,eps,variant", [
    ("poisson3d_20_leaf64_gc", lambda: pb.poisson(20, 3), 64, 1e-2, "gc"),
    ("lognormal2d_48_s2_leaf8_lorasp", lambda: pb.lognormal(48, 2, 2.0, 1002), 8, 1e-2, "lorasp"),
], ids=["poisson3d_20_leaf64_gc", "lognormal2d_48_s2_leaf8_lorasp"])
def test_colour_orders_match_oracle(name, make, leaf, eps, variant, order):
    """Both elimination orders inside a level (R8, opt.order) against the oracle run in the
    same order: equal schedules give equal ranks and z to the FP64 bar."""
    say("order", order, name)
    p = make()
    F = O.factor(p.row_ptr, p.col_idx, p.values, p.coords, leaf=leaf, eps=eps,
                 variant=O.GC if variant == "gc" else O.LORASP, order=order)
    F_, S, r, z_ref, z = run_pair(p, leaf, eps, variant, F=F, order=order)
    assert S.stats()["colours"] == sum(len(lev.colours) for lev in F.levels.values())
    check_parity(F, S, z, z_ref, f"{name}/{order}")
    S.close()
