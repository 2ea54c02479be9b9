"""The batched serving engine (se_server_create_batched): every resident solve
advanced one LOBPCG iteration per step with one launch per phase for all of
them. Results are checked against the FP64 oracle and the host-recomputed
stopping test, and bitwise alone against in a mix and with against without
the graph."""
import os

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import gpu_ctx

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return gpu_ctx()


def _x0(n, nb, seed):
    import torch

    return torch.from_numpy(np.ascontiguousarray(W.gaussian_block(n, nb, seed).T)).cuda()


def _serve(ctx, reqs, slots, strategy="fix", budget=16 << 30, stats=None, **kw):
    """Submit every (A, spec) at once; returns [(lam, V (n x n_ev), info)].
    stats: a list that receives the engine's (steps, graph_steps)."""
    import torch

    from paper_2409_05572_amd import api

    srv = api.Server(ctx, hbm_budget_bytes=budget, max_slots=slots, batched=True)
    try:
        out = []
        keep = []
        for A, s in reqs:
            M = api.Matrix.from_csr(ctx, A)
            x0 = _x0(A.n, s["n_ev"] + s["n_extra"], s["pot_seed"])
            torch.cuda.synchronize()
            keep.append((M, x0))
            out.append(srv.submit(M, x0, s["n_ev"], s["n_extra"], strategy=strategy, **kw))
        res = []
        for t, lam, V in out:
            info, _, _ = srv.wait(t)
            res.append((lam.cpu().numpy(), V.cpu().numpy().T, info))
        if stats is not None:
            stats.append(srv.batch_stats())
        return res
    finally:
        srv.close()


def _check_against_oracle(A, s, lam, V, info, strategy="fix"):
    import oracle as O
    from tests.gpu_util import cluster_angles

    assert info.converged, (s, info.iterations)
    S = A.to_scipy()
    R = O.solvers._apply(S, V) - V * lam[None, :]
    ratio = np.linalg.norm(R, axis=0) / (A.anorm * np.linalg.norm(V, axis=0))
    assert ratio.max() <= 1e-8 * 1.0001
    X0 = W.gaussian_block(A.n, s["n_ev"] + s["n_extra"], s["pot_seed"])
    se = O.SEParams(strategy) if strategy != "none" else None
    n_es = s["n_ev"] + min(5, s["n_extra"] - 1)
    ref = O.lobpcg(S, X0, s["n_ev"], A.anorm, tol=1e-8, n_es=n_es, se=se)
    assert ref.converged
    scale = np.maximum(np.abs(ref.lam), 1e-3 * A.anorm)
    assert np.max(np.abs(lam - ref.lam) / scale) <= 1e-10
    assert cluster_angles(lam, V, ref.V) <= 1e-6
    assert np.abs(V.T @ V - np.eye(s["n_ev"])).max() <= 1e-12
    # the same method from the same block: the iteration counts agree up to
    # the rounding-level drift of the trajectories
    assert abs(info.iterations - ref.iterations) <= max(3, 0.1 * ref.iterations), (info.iterations, ref.iterations)
    return ref


def test_one_request_matches_the_oracle(ctx):
    specs = W.serving_requests(1, seed=93, n_min=3e3, n_max=3e3, ev_min=8, ev_max=8)
    reqs = [(W.potential_laplacian(s["m"], s["dim"], 2.0, s["pot_seed"]), s) for s in specs]
    print("batched: one request", specs[0], flush=True)
    (lam, V, info), = _serve(ctx, reqs, 1)
    _check_against_oracle(*reqs[0], lam, V, info)


def test_served_stream_matches_the_oracle(ctx):
    """Serving-stream requests (2-D and 3-D Laplacians with a potential
    U[-2, 2], different n and n_ev), more requests than slots, so solves join
    at step boundaries while others run; shrink-and-expand (fix) on."""
    specs = W.serving_requests(6, seed=93, n_min=2e3, n_max=1.5e4, ev_min=4, ev_max=24)
    reqs = [(W.potential_laplacian(s["m"], s["dim"], 2.0, s["pot_seed"]), s) for s in specs]
    assert {s["dim"] for _, s in reqs} == {2, 3}
    print("batched: stream", [(A.n, s["n_ev"]) for A, s in reqs], flush=True)
    res = _serve(ctx, reqs, 3)
    shrinks = 0
    for (A, s), (lam, V, info) in zip(reqs, res):
        _check_against_oracle(A, s, lam, V, info)
        shrinks += info.n_shrinks
    assert shrinks > 0


@pytest.mark.parametrize("strategy", ["slope", "slopek", "none"])
def test_strategies_match_the_oracle(ctx, strategy):
    specs = W.serving_requests(3, seed=41, n_min=2e3, n_max=8e3, ev_min=6, ev_max=20)
    reqs = [(W.potential_laplacian(s["m"], s["dim"], 2.0, s["pot_seed"]), s) for s in specs]
    print("batched: strategy", strategy, flush=True)
    res = _serve(ctx, reqs, 3, strategy=strategy)
    for (A, s), (lam, V, info) in zip(reqs, res):
        _check_against_oracle(A, s, lam, V, info, strategy=strategy)


def test_results_identical_alone_and_in_the_mix(ctx):
    specs = W.serving_requests(5, seed=57, n_min=2e3, n_max=1.2e4, ev_min=4, ev_max=20)
    reqs = [(W.potential_laplacian(s["m"], s["dim"], 2.0, s["pot_seed"]), s) for s in specs]
    print("batched: alone vs mix", flush=True)
    mix = _serve(ctx, reqs, 4)
    for q, r in enumerate(reqs):
        (lam, V, info), = _serve(ctx, [r], 1)
        assert np.array_equal(lam, mix[q][0]) and np.array_equal(V, mix[q][1])
        assert info.iterations == mix[q][2].iterations


def test_graph_and_direct_launches_agree_bitwise(ctx):
    specs = W.serving_requests(3, seed=61, n_min=2e3, n_max=6e3, ev_min=4, ev_max=16)
    reqs = [(W.potential_laplacian(s["m"], s["dim"], 2.0, s["pot_seed"]), s) for s in specs]
    print("batched: graph vs direct", flush=True)
    st = []
    os.environ["SE_BATCH_GRAPH"] = "1"
    try:
        with_graph = _serve(ctx, reqs, 3, stats=st)
    finally:
        del os.environ["SE_BATCH_GRAPH"]
    direct = _serve(ctx, reqs, 3, stats=st)
    # every step of the first server replayed the graph, none of the second
    assert st[0][0] > 0 and st[0][1] == st[0][0] and st[1][0] > 0 and st[1][1] == 0, st
    for a, b in zip(with_graph, direct):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_unsupported_and_oversized_requests(ctx):
    import torch

    from paper_2409_05572_amd import api
    from paper_2409_05572_amd._lib import SeError

    A = W.potential_laplacian(40, 2, 2.0, 3)
    M = api.Matrix.from_csr(ctx, A)
    srv = api.Server(ctx, hbm_budget_bytes=1 << 30, max_slots=2, batched=True)
    try:
        x0 = _x0(A.n, 12, 1)
        torch.cuda.synchronize()
        for kw in (dict(solver="si"), dict(precision="fp32"), dict(precond="jacobi")):
            with pytest.raises(SeError) as e:
                srv.submit(M, x0, 8, 4, **kw)
            assert e.value.status == -6
        with pytest.raises(SeError) as e:
            srv.submit(M, _x0(A.n, 100, 1), 80, 20)
        assert e.value.status == -6
    finally:
        srv.close()
    tiny = api.Server(ctx, hbm_budget_bytes=1 << 20, max_slots=2, batched=True)
    try:
        with pytest.raises(SeError) as e:
            tiny.submit(M, x0, 8, 4)
        assert e.value.status == -5
    finally:
        tiny.close()


def test_tight_budget_runs_requests_one_at_a_time(ctx):
    from paper_2409_05572_amd import api

    specs = W.serving_requests(3, seed=71, n_min=4e3, n_max=4e3, ev_min=8, ev_max=8)
    reqs = [(W.potential_laplacian(s["m"], s["dim"], 2.0, s["pot_seed"]), s) for s in specs]
    fp = max(api.lib().se_batched_footprint(A.n, s["n_ev"], s["n_extra"]) for A, s in reqs)
    print("batched: tight budget", fp, flush=True)
    res = _serve(ctx, reqs, 3, budget=int(fp * 1.5))
    alone = [_serve(ctx, [r], 1)[0] for r in reqs]
    for a, b in zip(res, alone):
        assert a[2].converged and np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_widest_block_matches_the_oracle(ctx):
    """nb = 96, the engine's limit: the gathered W block reaches past 112
    columns after an expansion (the global-memory Cholesky-QR transform) and
    the Rayleigh-Ritz order reaches 288 (the register tridiagonalization of
    the trailing 192 reflectors after the leading ones in L2)."""
    s = {"dim": 3, "m": 16, "n": 16 ** 3, "n_ev": 64, "n_extra": 32, "pot_seed": 10077}
    A = W.potential_laplacian(s["m"], s["dim"], 2.0, s["pot_seed"])
    print("batched: nb = 96", flush=True)
    (lam, V, info), = _serve(ctx, [(A, s)], 2)
    assert info.n_shrinks > 0 and info.n_expands > 0
    _check_against_oracle(A, s, lam, V, info)
