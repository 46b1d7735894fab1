"""C-ABI library checks that need no GPU: it loads, exports every declared symbol, and its
host symbolic analysis (bisection, adjacency, simulated fill, colour order) produces
exactly the integer schedule of the CPU oracle, which implements the same rules separately.
"""
import ctypes

import numpy as np
import pytest

import oracle as O
from paper_1611_03189_amd import hsolve as H
from paper_1611_03189_amd import problems as pb


@pytest.fixture(scope="module")
def lib():
    return H.load()


def test_library_exports_every_declared_symbol(lib):
    names = H.exported_names()
    assert "hsolve_analyze" in names and "hsolve_factor" in names
    assert "hsolve_apply" in names and "hsolve_solve" in names
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for code, name in H.STATUS.items():
        assert lib.hsolve_status_string(code).decode() == name


CASES = [
    ("poisson2d_32_leaf16", lambda: pb.poisson(32, 2), 16, 1e-2, "gc"),
    ("poisson2d_24_leaf8", lambda: pb.poisson(24, 2), 8, 0.1, "lorasp"),
    ("lognormal2d_32_leaf8", lambda: pb.lognormal(32, 2, 2.0, 3), 8, 1e-2, "gc"),
    ("poisson3d_12_leaf16", lambda: pb.poisson(12, 3), 16, 1e-2, "gc"),
    ("poisson3d_16_leaf64", lambda: pb.poisson(16, 3), 64, 1e-2, "gc"),
    ("chain_100_leaf5", lambda: pb.chain(100), 5, 0.1, "gc"),
    ("poisson2d_20_nocoords", lambda: pb.poisson(20, 2), 8, 1e-2, "gc"),
]


@pytest.mark.parametrize("order", ["waiting", "index"])
@pytest.mark.parametrize("neighbours", ["footprint", "geometric"])
@pytest.mark.parametrize("name,make,leaf,eps,variant", CASES, ids=[c[0] for c in CASES])
def test_schedule_matches_oracle(name, make, leaf, eps, variant, neighbours, order):
    p = make()
    coords = None if name.endswith("nocoords") else p.coords
    F = O.factor(p.row_ptr, p.col_idx, p.values, coords, leaf=leaf, eps=eps,
                 variant=O.GC if variant == "gc" else O.LORASP, neighbours=neighbours, order=order)
    with H.HSolver(p.row_ptr, p.col_idx, coords=coords, leaf=leaf, eps=eps, variant=variant,
                   neighbours=neighbours, order=order) as S:
        assert S.depth == F.L
        perm, off = S.leaf_order()
        assert np.array_equal(perm, np.concatenate(F.leaves))
        assert np.array_equal(np.diff(off), [len(c) for c in F.leaves])
        for d, lev in F.levels.items():
            col, nc = S.colours(d)
            assert nc == len(lev.colours)
            for ci, members in enumerate(lev.colours):
                assert sorted(np.nonzero(col == ci)[0].tolist()) == members
            for s, nf in lev.nodes.items():
                nb, ws = S.node_sets(d, s)
                exp_nb = [2 * n + (st == "R") for (n, st, _) in nf.nbrs]
                exp_ws = [2 * w + (st == "R") for w, st in zip(nf.W, nf.Wstate)]
                assert nb.tolist() == exp_nb, (d, s)
                assert ws.tolist() == exp_ws, (d, s)
            # nodes the oracle never eliminated (empty) have no colour in the library
            empty = set(range(1 << d)) - set(lev.nodes)
            assert all(col[e] == -1 for e in empty)


def test_analyze_rejects_bad_input(lib):
    p = pb.poisson(6, 2)
    with pytest.raises(H.HSolveError) as e:
        H.HSolver(p.row_ptr, p.col_idx[::-1].copy(), coords=p.coords)
    assert e.value.status == -1                      # unsorted rows
    rp, ci = p.row_ptr.copy(), p.col_idx.copy()
    assert ci[:3].tolist() == [0, 1, 6]
    ci[2] = 7                                        # (0,7) without (7,0); row 0 stays sorted
    with pytest.raises(H.HSolveError) as e:
        H.HSolver(rp, ci, coords=p.coords)
    assert e.value.status == -2
    with pytest.raises(H.HSolveError) as e:
        H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, eps=-1.0)
    assert e.value.status == -1
    bad = p.col_idx.copy()
    bad[-1] = p.n + 5
    with pytest.raises(H.HSolveError):
        H.HSolver(p.row_ptr, bad, coords=p.coords)
    # first super nodes (pairs of leaves) above the 512 the kernels take: rejected by the analysis
    big = pb.poisson(16, 3)
    with pytest.raises(H.HSolveError) as e:
        H.HSolver(big.row_ptr, big.col_idx, coords=big.coords, leaf=600)
    assert e.value.status == -1
    H.HSolver(big.row_ptr, big.col_idx, coords=big.coords, leaf=256).close()   # pairs of 512
    for kw in ({"apply_prec": 16}, {"krylov": 4}, {"krylov": "gmres", "restart": 0}):
        with pytest.raises(H.HSolveError) as e:
            H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, **kw)
        assert e.value.status == -1, kw


def test_options_accept_solver_variants(lib):
    p = pb.poisson(6, 2)
    for kw in ({"apply_prec": 32, "krylov": "fpcg"}, {"krylov": "gmres", "restart": 30},
               {"apply_prec": 64, "krylov": "pcg"}, {"overlap_pivots": False}, {"krylov": "stationary"}):
        with H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, **kw) as S:
            assert S._h


def test_state_errors_without_factor(lib):
    p = pb.poisson(6, 2)
    with H.HSolver(p.row_ptr, p.col_idx, coords=p.coords) as S:
        dummy = ctypes.c_void_p(1)
        assert lib.hsolve_apply(S._h, 1, dummy, p.n, dummy, p.n) == -6
        assert lib.hsolve_solve(S._h, 1, dummy, p.n, dummy, p.n, None) == -6
        assert lib.hsolve_ranks(S._h, 0, np.zeros(1, np.int32).ctypes.data_as(
            ctypes.POINTER(ctypes.c_int32))) == -6


def test_new_options_are_checked(lib):
    p = pb.poisson(6, 2)
    for kw in ({"factor_prec": 16}, {"max_super": 0}, {"max_super": 513}, {"max_nrhs": 0},
               {"eps_schedule": 3}, {"cmp_lpe": 3}, {"cmp_lpe": 128}, {"cmp_vectors": 3},
               {"variant": 3}, {"eps1": -0.1}, {"eps1": 1.0}, {"neighbours": 2}, {"cmp_ritz": 2},
               {"order": 2}, {"order": -1}):
        with pytest.raises(H.HSolveError) as e:
            H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, **kw)
        assert e.value.status == -1, kw
    for kw in ({"eps_schedule": "shrink"}, {"eps_schedule": "grow"}, {"cmp_lpe": 8, "cmp_vectors": 1},
               {"cmp_lpe": 1, "cmp_vectors": 2}, {"max_super": 64, "max_nrhs": 4},
               {"variant": "gc_proj1", "eps1": 1e-2}, {"neighbours": "geometric"},
               {"factor_prec": 32, "krylov": "fpcg"}, {"cmp_ritz": False}, {"order": "index"}):
        with H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, **kw) as S:
            assert S.arena_bound > 0


def test_arena_bound_is_monotone_in_the_caps(lib):
    """The analysis replays the factorization with every rank at its largest value; a lower
    super-node cap or fewer right-hand sides can only shrink that replay."""
    p = pb.poisson(16, 3)
    bounds = []
    for ms in (512, 256, 128):
        with H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=16, eps=1e-2, max_super=ms) as S:
            bounds.append(S.arena_bound)
    assert bounds[0] >= bounds[1] >= bounds[2] > 0
    with H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=16, max_nrhs=1) as S1, \
            H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=16, max_nrhs=256) as S2:
        assert S1.arena_bound <= S2.arena_bound
        # at least the CSR pattern and values, and the first level's dense diagonal blocks
        L = S1.depth
        _, off = S1.leaf_order()
        diag = sum(8 * (off[2 * s + 2] - off[2 * s]) ** 2 for s in range(1 << (L - 1)))
        assert S1.arena_bound >= 12 * p.nnz + diag


def test_arena_too_small_or_misaligned_is_rejected_before_gpu_work(lib):
    """The arena checks run on the host before any device call: a too-small arena gives
    HSOLVE_ERR_OOM, a misaligned one HSOLVE_ERR_INVALID, and the plan stays unfactored."""
    p = pb.poisson(8, 2)
    with H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=8) as S:
        vals = np.ascontiguousarray(p.values)
        fake = ctypes.c_void_p(1 << 40)                  # never dereferenced
        assert lib.hsolve_factor(S._h, vals.ctypes.data_as(ctypes.c_void_p), fake, 4096) == -4
        assert b"arena too small" in lib.hsolve_last_error(S._h)
        assert lib.hsolve_factor(S._h, vals.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p((1 << 40) + 8),
                                 S.arena_bound) == -1
        assert lib.hsolve_factor(S._h, vals.ctypes.data_as(ctypes.c_void_p), None, S.arena_bound) == -1
        dummy = ctypes.c_void_p(1)
        assert lib.hsolve_apply(S._h, 1, dummy, p.n, dummy, p.n) == -6


def test_binding_checks_shapes_before_the_library(lib):
    """Sizes the C ABI cannot see (it takes no lengths) are checked in the binding."""
    torch = pytest.importorskip("torch")
    p = pb.poisson(6, 2)
    with H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=8) as S:
        with pytest.raises(ValueError):
            S.factor(np.ones(p.nnz - 1))
        if not torch.cuda.is_available():
            return
        with pytest.raises(ValueError):
            S.apply(torch.ones(p.n - 1, dtype=torch.float64, device="cuda"))
