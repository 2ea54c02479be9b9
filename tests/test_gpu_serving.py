"""The serving runtime (se_server_*) on the GPU: admission by HBM footprint,
results identical to a lone se_solve, queueing under a tight budget."""
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


def _requests():
    specs = W.serving_requests(7, seed=77, n_min=2e3, n_max=4e4, ev_min=4, ev_max=24)
    return [(W.potential_laplacian(s["m"], s["dim"], 2.0, s["pot_seed"]), s) for s in specs]


def test_footprint_covers_the_workspace_of_a_solve(ctx):
    from paper_2409_05572_amd import api

    for prec in ("fp64", "fp32"):
        c = api.Context(0)  # fresh workspace
        A = W.potential_laplacian(30, 2, 2.0, 5)
        M = api.Matrix.from_csr(c, A)
        _, _, info = api.solve(c, M, _x0(A.n, 12, 3), 8, 4, strategy="fix", precision=prec)
        fp = api.footprint(A.n, A.nnz, 8, 4, precision=prec)
        assert info.workspace_bytes <= fp <= 1.3 * info.workspace_bytes + (1 << 20)


@pytest.mark.parametrize("solver,opts", [("si", dict(filter_degree=4, expand_vectors="powered")),
                                         ("tracemin", {}), ("lobpcg", dict(precond="jacobi")),
                                         ("sd", dict(precond="jacobi"))])
def test_footprint_covers_every_solver(ctx, solver, opts):
    from paper_2409_05572_amd import api

    c = api.Context(0)  # fresh workspace
    A = W.laplacian_3d(14)
    M = api.Matrix.from_csr(c, A)
    _, _, info = api.solve(c, M, _x0(A.n, 12, 3), 8, 4, strategy="fix", solver=solver, max_iter=4000, **opts)
    fp = api.footprint(A.n, A.nnz, 8, 4, solver=solver)
    assert info.workspace_bytes <= fp <= 1.3 * info.workspace_bytes + (1 << 20)


def test_results_identical_alone_and_in_the_mix(ctx):
    import torch

    from paper_2409_05572_amd import api

    reqs = _requests()
    mats = [api.Matrix.from_csr(ctx, A) for A, _ in reqs]
    alone = []
    for M, (A, s) in zip(mats, reqs):
        lam, V, info = api.solve(ctx, M, _x0(A.n, s["n_ev"] + s["n_extra"], s["pot_seed"]), s["n_ev"],
                                 s["n_extra"], strategy="fix")
        assert info.converged
        alone.append((lam.cpu().numpy(), V.cpu().numpy()))
    srv = api.Server(ctx, hbm_budget_bytes=64 << 30, max_slots=3)
    try:
        tickets = []
        for M, (A, s) in zip(mats, reqs):
            x0 = _x0(A.n, s["n_ev"] + s["n_extra"], s["pot_seed"])
            torch.cuda.synchronize()
            tickets.append(srv.submit(M, x0, s["n_ev"], s["n_extra"], strategy="fix"))
        for (t, lam, V), (lam0, V0) in zip(tickets, alone):
            info, q_ms, run_ms = srv.wait(t)
            assert info.converged and info.max_stop_ratio <= 1e-8 and run_ms > 0 and q_ms >= 0
            assert np.array_equal(lam.cpu().numpy(), lam0) and np.array_equal(V.cpu().numpy(), V0)
    finally:
        srv.close()


def test_tight_budget_queues_and_oversized_request_is_rejected(ctx):
    import torch

    from paper_2409_05572_amd import api
    from paper_2409_05572_amd._lib import SeError

    reqs = _requests()[:4]
    fps = [api.footprint(A.n, A.nnz, s["n_ev"], s["n_extra"]) for A, s in reqs]
    budget = int(max(fps) * 1.05)  # room for one request at a time (slots keep their workspace)
    srv = api.Server(ctx, hbm_budget_bytes=budget, max_slots=4)
    try:
        mats = [api.Matrix.from_csr(ctx, A) for A, _ in reqs]
        tickets = []
        for M, (A, s) in zip(mats, reqs):
            x0 = _x0(A.n, s["n_ev"] + s["n_extra"], s["pot_seed"])
            torch.cuda.synchronize()
            tickets.append(srv.submit(M, x0, s["n_ev"], s["n_extra"]))
        waits = [srv.wait(t[0]) for t in tickets]
        assert all(w[0].converged for w in waits)
        assert max(w[1] for w in waits[1:]) > 0.0  # later requests waited for memory
        big = W.potential_laplacian(60, 3, 2.0, 1)
        Mb = api.Matrix.from_csr(ctx, big)
        with pytest.raises(SeError):
            srv.submit(Mb, _x0(big.n, 48, 1), 32, 16)
    finally:
        srv.close()


def test_mixed_precision_requests_share_the_server(ctx):
    import torch

    from paper_2409_05572_amd import api

    reqs = _requests()[:4]
    srv = api.Server(ctx, hbm_budget_bytes=32 << 30, max_slots=2)
    try:
        out = []
        for i, (A, s) in enumerate(reqs):
            M = api.Matrix.from_csr(ctx, A)
            x0 = _x0(A.n, s["n_ev"] + s["n_extra"], s["pot_seed"])
            torch.cuda.synchronize()
            out.append((M, x0, srv.submit(M, x0, s["n_ev"], s["n_extra"], strategy="fix",
                                          precision="fp32" if i % 2 else "fp64")))
        for M, x0, (t, lam, V) in out:
            info, _, _ = srv.wait(t)
            assert info.converged and info.max_stop_ratio <= 1e-8
    finally:
        srv.close()


def test_destroy_with_queued_requests_returns(ctx):
    import torch

    from paper_2409_05572_amd import api

    reqs = _requests()[:3]
    srv = api.Server(ctx, hbm_budget_bytes=64 << 30, max_slots=1)
    keep = []
    for A, s in reqs:
        M = api.Matrix.from_csr(ctx, A)
        x0 = _x0(A.n, s["n_ev"] + s["n_extra"], s["pot_seed"])
        torch.cuda.synchronize()
        keep.append((M, x0, srv.submit(M, x0, s["n_ev"], s["n_extra"])))
    srv.close()  # finishes the running solve, drops the queued ones
    torch.cuda.synchronize()


def test_every_solver_served_identically_to_a_lone_solve(ctx):
    """Requests for each solver and option (Chebyshev-filtered SI with a
    powered X_drop, TraceMIN, Jacobi-preconditioned LOBPCG, SD with random
    expansions) share the server and return bitwise what a lone se_solve
    returns."""
    import torch

    from paper_2409_05572_amd import api

    A = W.laplacian_3d(16)  # positive definite (TraceMIN needs it)
    M = api.Matrix.from_csr(ctx, A)
    opts = [dict(solver="si", filter_degree=6, expand_vectors="powered"), dict(solver="tracemin"),
            dict(solver="lobpcg", precond="jacobi"), dict(solver="sd", expand_vectors="random", seed=5)]
    alone = []
    for i, o in enumerate(opts):
        lam, V, info = api.solve(ctx, M, _x0(A.n, 16, 40 + i), 10, 6, strategy="fix", n_es=12,
                                 max_iter=4000, **o)
        assert info.converged, o
        alone.append((lam.cpu().numpy(), V.cpu().numpy()))
    srv = api.Server(ctx, hbm_budget_bytes=16 << 30, max_slots=4)
    try:
        tickets = []
        for i, o in enumerate(opts):
            x0 = _x0(A.n, 16, 40 + i)
            torch.cuda.synchronize()
            tickets.append(srv.submit(M, x0, 10, 6, strategy="fix", n_es=12, max_iter=4000, **o))
        for (t, lam, V), (lam0, V0), o in zip(tickets, alone, opts):
            info, _, _ = srv.wait(t)
            assert info.converged, o
            assert np.array_equal(lam.cpu().numpy(), lam0) and np.array_equal(V.cpu().numpy(), V0), o
    finally:
        srv.close()


def test_idle_workspace_is_released_for_a_larger_request(ctx):
    """Two small requests run at once and leave both slots holding workspace;
    a larger request then fits the budget only if the other idle slot gives
    its workspace back. It must start (no wait on memory only idle slots
    hold) and converge."""
    import time

    import torch

    import oracle as O
    from paper_2409_05572_amd import api

    small = [W.potential_laplacian(40, 2, 2.0, s) for s in (1, 2)]
    big = W.potential_laplacian(56, 2, 2.0, 3)
    fs = api.footprint(small[0].n, small[0].nnz, 8, 4)
    fb = api.footprint(big.n, big.nnz, 8, 4)
    budget = int(2.05 * fs)
    assert fs < fb <= budget < fs + fb
    srv = api.Server(ctx, hbm_budget_bytes=budget, max_slots=2)
    try:
        keep = []
        for i, A in enumerate(small):
            M = api.Matrix.from_csr(ctx, A)
            x0 = _x0(A.n, 12, 10 + i)
            torch.cuda.synchronize()
            keep.append((M, x0, srv.submit(M, x0, 8, 4)))
        for _, _, (t, _, _) in keep:
            assert srv.wait(t)[0].converged
        Mb = api.Matrix.from_csr(ctx, big)
        xb = _x0(big.n, 12, 12)
        torch.cuda.synchronize()
        t, lam, V = srv.submit(Mb, xb, 8, 4)
        deadline = time.monotonic() + 60.0
        while not srv.poll(t):
            assert time.monotonic() < deadline, "request waited on workspace held by idle slots"
            time.sleep(0.01)
        info, _, _ = srv.wait(t)
        assert info.converged
        lam, V = lam.cpu().numpy(), V.cpu().numpy().T
        R = big.to_scipy() @ V - V * lam[None, :]
        ratio = np.linalg.norm(R, axis=0) / (big.anorm * np.linalg.norm(V, axis=0))
        assert ratio.max() <= 1e-8
        ref = O.lobpcg(big.to_scipy(), W.gaussian_block(big.n, 12, 12), 8, big.anorm, tol=1e-8)
        scale = np.maximum(np.abs(ref.lam), 1e-3 * big.anorm)
        assert np.max(np.abs(lam - ref.lam) / scale) <= 1e-10
    finally:
        srv.close()


def test_served_results_match_the_oracle(ctx):
    """Requests of the serving stream's kind (2-D and 3-D Laplacians with a
    potential U[-2, 2], different n and n_ev) served together, each checked on
    its own: the stopping test recomputed on the host with the oracle's
    product, the eigenvalues against the FP64 oracle started from the same
    block (error relative to max(|lambda|, 1e-3 ||A||)), the eigenvectors
    through principal angles of complete clusters, orthonormality."""
    import torch

    import oracle as O
    from paper_2409_05572_amd import api
    from tests.gpu_util import cluster_angles

    specs = W.serving_requests(5, seed=93, n_min=2e3, n_max=1.5e4, ev_min=4, ev_max=20)
    reqs = [(W.potential_laplacian(s["m"], s["dim"], 2.0, s["pot_seed"]), s) for s in specs]
    assert {s["dim"] for _, s in reqs} == {2, 3}
    srv = api.Server(ctx, hbm_budget_bytes=16 << 30, max_slots=3)
    try:
        out = []
        for A, s in reqs:
            M = api.Matrix.from_csr(ctx, A)
            x0 = _x0(A.n, s["n_ev"] + s["n_extra"], s["pot_seed"])
            torch.cuda.synchronize()
            out.append((A, s, M, x0, srv.submit(M, x0, s["n_ev"], s["n_extra"], strategy="fix")))
        for A, s, M, x0, (t, lam, V) in out:
            info, _, _ = srv.wait(t)
            assert info.converged
            lam, V = lam.cpu().numpy(), V.cpu().numpy().T
            S = A.to_scipy()
            R = O.solvers._apply(S, V) - V * lam[None, :]
            ratio = np.linalg.norm(R, axis=0) / (A.anorm * np.linalg.norm(V, axis=0))
            assert ratio.max() <= 1e-8 * 1.0001
            X0 = W.gaussian_block(A.n, s["n_ev"] + s["n_extra"], s["pot_seed"])
            ref = O.lobpcg(S, X0, s["n_ev"], A.anorm, tol=1e-8)
            scale = np.maximum(np.abs(ref.lam), 1e-3 * A.anorm)
            assert np.max(np.abs(lam - ref.lam) / scale) <= 1e-10
            assert cluster_angles(lam, V, ref.V) <= 1e-6
            assert np.abs(V.T @ V - np.eye(s["n_ev"])).max() <= 1e-12
    finally:
        srv.close()
