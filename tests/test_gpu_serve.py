"""Request loop (continuous batching over several HIP streams): every request gives the same
bits alone and in the mix, and every result reaches the 1e-10 relative residual."""
import numpy as np
import pytest

from paper_1611_03189_amd import problems as pb

pytestmark = pytest.mark.gpu


def say(name):
    print(f"\n[case] {name}", flush=True)


def _requests():
    from paper_1611_03189_amd.serve import Request
    out = []
    for i, (dim, N, nrhs) in enumerate([(2, 40, 2), (3, 12, 1), (2, 56, 3), (3, 14, 2), (2, 24, 1), (3, 10, 4)]):
        p = pb.lognormal(N, dim, 1.0, 300 + i)
        b = pb.rhs(p.n, nrhs, 400 + i)
        out.append(Request(i, p.row_ptr, p.col_idx, p.values, p.coords, b, leaf=16 if dim == 2 else 64,
                           eps=1e-2))
    return out


def test_request_loop_results_equal_alone_and_in_mix():
    say("serve_alone_vs_mix")
    import torch
    from paper_1611_03189_amd.serve import RequestLoop
    reqs = _requests()
    alone = RequestLoop(slots=1).run(reqs, realtime=False)
    mix = RequestLoop(slots=4).run(reqs, realtime=False)
    assert [r.rid for r in alone.results] == [r.rid for r in mix.results] == list(range(len(reqs)))
    for q, a, m in zip(reqs, alone.results, mix.results):
        assert np.array_equal(a.x, m.x), f"request {q.rid} differs in the mix"
        assert a.iterations == m.iterations and a.converged and m.converged
        import scipy.sparse as sp
        A = sp.csr_matrix((q.values, q.col_idx, q.row_ptr), shape=(q.n, q.n))
        res = np.linalg.norm(q.b - A @ m.x, axis=0) / np.linalg.norm(q.b, axis=0)
        assert np.all(res <= 2e-10), res
    # the mix ran requests on several slots at once
    overlap = any(x.slot != y.slot and x.t_start < y.t_done and y.t_start < x.t_done
                  for x in mix.results for y in mix.results)
    assert overlap
    st = mix.stats()
    assert st["requests"] == len(reqs) and st["all_converged"] and st["p99_ms"] >= st["p50_ms"] > 0


def test_request_loop_admission_respects_budget():
    # a budget that fits one request at a time still completes every request
    say("serve_budget")
    from paper_1611_03189_amd.serve import RequestLoop
    reqs = _requests()[:3]
    loop = RequestLoop(slots=3, memory_budget=1)
    out = loop.run(reqs, realtime=False)
    assert len(out.results) == 3 and all(r.converged for r in out.results)
    spans = sorted((r.t_start, r.t_done) for r in out.results)
    assert all(spans[i][1] <= spans[i + 1][0] + 1e-6 for i in range(len(spans) - 1))


def test_request_loop_mixed_precision_alone_and_in_mix():
    """The served mixed form (FP32 factorization, FP64 flexible PCG): the same bits alone and in
    the mix, every result at the 1e-10 true residual."""
    say("serve_mixed")
    import scipy.sparse as sp
    from paper_1611_03189_amd.serve import RequestLoop
    reqs = _requests()
    alone = RequestLoop(slots=1, mixed=True).run(reqs, realtime=False)
    mix = RequestLoop(slots=4, mixed=True).run(reqs, realtime=False)
    for q, a, m in zip(reqs, alone.results, mix.results):
        assert np.array_equal(a.x, m.x) and a.converged and m.converged
        A = sp.csr_matrix((q.values, q.col_idx, q.row_ptr), shape=(q.n, q.n))
        res = np.linalg.norm(q.b - A @ m.x, axis=0) / np.linalg.norm(q.b, axis=0)
        assert np.all(res <= 2e-10), res
