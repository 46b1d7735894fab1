"""The apply's sweeps replayed as a captured HIP graph give the same bits as the launches
issued one by one: several replays of one graph, with other eager GPU work and host
synchronisations between them, each checked against the eager result; PCG and the FP32
solve phase through the graph; a refactorization drops the captured graphs."""
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


@pytest.mark.parametrize("apply_prec,nrhs", [(64, 1), (64, 3), (32, 2), (64, 8), (32, 6)])
def test_graph_replays_equal_eager(apply_prec, nrhs):
    say("graph replays", apply_prec, nrhs)
    p = pb.poisson(14, 3)
    kw = dict(coords=p.coords, leaf=16, eps=1e-2, apply_prec=apply_prec)
    Sg = H.HSolver(p.row_ptr, p.col_idx, apply_graph=True, **kw)
    Se = H.HSolver(p.row_ptr, p.col_idx, apply_graph=False, **kw)
    v = torch.from_numpy(p.values).cuda()
    Sg.factor(v)
    Se.factor(v)
    other = pb.poisson(20, 2)
    So = H.HSolver(other.row_ptr, other.col_idx, coords=other.coords, leaf=8, eps=1e-2, apply_graph=False)
    So.factor(torch.from_numpy(other.values).cuda())
    for rep in range(4):
        R = torch.from_numpy(np.ascontiguousarray(pb.rhs(p.n, nrhs, 100 + rep))).cuda()
        zg = Sg.apply(R)
        So.apply(torch.ones(other.n, dtype=torch.float64, device="cuda"))     # eager work between replays
        _ = Sg.spmv(torch.ones(p.n, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        ze = Se.apply(R)
        assert torch.equal(zg, ze), rep
    b = torch.from_numpy(pb.rhs(p.n, 1, 7)[:, 0]).cuda()
    xg, stg = Sg.solve(b)
    xe, ste = Se.solve(b)
    assert torch.equal(xg, xe) and stg["iterations"] == ste["iterations"]
    # a refactorization with other values: the replayed sweeps follow the new factor
    v2 = torch.from_numpy(pb.lognormal(14, 3, 1.0, 5).values).cuda()
    Sg.factor(v2)
    Se.factor(v2)
    R = torch.from_numpy(np.ascontiguousarray(pb.rhs(p.n, nrhs, 9))).cuda()
    assert torch.equal(Sg.apply(R), Se.apply(R))
    for S in (Sg, Se, So):
        S.close()


def test_every_gemm_tile_shape_gives_the_same_bits():
    """The grouped GEMM adds each output's k products in the same order in every tile shape,
    so forcing any shape for every size bucket leaves the factorization bitwise unchanged."""
    say("gemm tile shapes")
    p = pb.lognormal(16, 3, 1.0, 3)
    r = torch.from_numpy(np.ascontiguousarray(pb.rhs(p.n, 2, 5))).cuda()
    v = torch.from_numpy(p.values).cuda()
    out = []
    try:
        for shape in range(len(H.GEMM_SHAPES)):
            H.set_gemm_choice([shape] * H.GEMM_BUCKETS)
            S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=32, eps=1e-2)
            S.factor(v)
            out.append(S.apply(r))
            S.close()
    finally:
        H.set_gemm_choice([0] * H.GEMM_BUCKETS)
    for z in out[1:]:
        assert torch.equal(z, out[0])


def test_autotuner_picks_a_shape_per_bucket():
    say("gemm autotune")
    res = H.tune_gemm()
    try:
        assert len(res["choice"]) == H.GEMM_BUCKETS
        assert all(0 <= c < len(H.GEMM_SHAPES) for c in res["choice"])
        ms = np.array(res["ms"])
        assert ms.shape == (H.GEMM_BUCKETS, len(H.GEMM_SHAPES)) and np.all(ms > 0)
        # the choice is the fastest timing of its bucket
        assert all(ms[b, res["choice"][b]] == ms[b].min() for b in range(H.GEMM_BUCKETS))
    finally:
        H.set_gemm_choice([0] * H.GEMM_BUCKETS)
