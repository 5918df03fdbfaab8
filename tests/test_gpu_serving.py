"""The request server (rqlp_server_*): requests admitted while others run,
under an HBM budget that forces queueing, each give bitwise the result of the
same request run alone, and the served results match the oracle."""
import numpy as np
import pytest
import torch

import oracle
from oracle.metrics import recon_diff, orth_error
import workloads
from tests.gpu_util import announce, to_dev, to_np

pytestmark = pytest.mark.gpu


def _requests(count, seed):
    reqs = workloads.serving_requests(count, seed, m_range=(64, 1200), n_range=(40, 700), kmax=100)
    As = [to_dev(workloads.request_matrix(r, np.float32)) for r in reqs]
    return reqs, As


def _outs(reqs, dev):
    return [(torch.empty((r["m"], r["k"] + r["p"]), device=dev), torch.empty((r["k"] + r["p"],) * 2, device=dev),
             torch.empty((r["n"], r["k"] + r["p"]), device=dev)) for r in reqs]


def test_same_alone_and_in_the_mix(gpu_lib):
    announce("serving: alone vs in the mix")
    reqs, As = _requests(24, 21)
    dev = As[0].device
    q = 1
    solo = [tuple(x.clone() for x in gpu_lib.decompose(A, r["k"], r["p"], q, seed=100 + i))
            for i, (r, A) in enumerate(zip(reqs, As))]
    torch.cuda.synchronize()
    sizes = [gpu_lib.server_request_bytes(r["m"], r["n"], r["k"], r["p"], q) for r in reqs]
    assert min(sizes) > 0
    budget = 3 * max(sizes)  # at most three requests' workspaces at a time
    srv = gpu_lib.Server(budget, slots=4)
    outs = _outs(reqs, dev)
    for o in outs:
        for x in o:
            x.fill_(float("nan"))
    torch.cuda.synchronize()
    pending, tickets, done = list(range(len(reqs))), {}, set()
    max_inflight = 0
    while len(done) < len(reqs):
        for _ in range(3):  # arrivals trickle in while earlier requests run
            if pending:
                i = pending.pop(0)
                tickets[srv.submit(As[i], reqs[i]["k"], reqs[i]["p"], q, 100 + i, outs[i])] = i
        fin, inflight, queued = srv.poll()
        max_inflight = max(max_inflight, inflight)
        done.update(fin)
    srv.close()
    assert max_inflight >= 2  # requests really overlapped
    assert not srv.failed
    for t, i in tickets.items():
        for a, b in zip(outs[i], solo[i]):
            assert torch.equal(a, b), f"request {i} differs from its solo run"
    # served results against the oracle (the reconstruction is unique even
    # where a request's matrix has rank below d)
    for i in (0, 5, 11, 23):
        r = reqs[i]
        A64 = to_np(As[i])
        Qg, Lg, Vg = (to_np(x) for x in outs[i])
        Qo, Lo, Vo = oracle.ruqlp(A64, r["k"], r["p"], q, 100 + i, omega_dtype="f32")
        delta = recon_diff(Qg, Lg, Vg, Qo, Lo, Vo) / np.linalg.norm(A64)
        d = r["k"] + r["p"]
        print(f"served request {i} ({r['m']}x{r['n']}, d={d}): Delta = {delta:.3e}", flush=True)
        assert delta <= 1e-5
        assert orth_error(Qg) <= 16 * np.sqrt(d) * 2.0 ** -24 and orth_error(Vg) <= 16 * np.sqrt(d) * 2.0 ** -24
        assert np.all(np.triu(Lg, 1) == 0.0) and np.all(np.diag(Lg) >= 0.0)


def test_submit_waits_for_the_callers_stream(gpu_lib):
    """A request's launches wait for the work enqueued on the submitting
    stream before submit: here A is written on a side stream, behind a
    chain of large products, and submitted from that stream with no host
    synchronization; the result is still the one of the final A."""
    announce("serving: submit orders after the caller's stream")
    reqs, As = _requests(1, 33)
    r, A = reqs[0], As[0]
    q = 1
    solo = tuple(x.clone() for x in gpu_lib.decompose(A, r["k"], r["p"], q, seed=7))
    torch.cuda.synchronize()
    A_late = torch.full_like(A, float("nan"))
    big = torch.randn(4096, 4096, device=A.device)
    out = _outs([r], A.device)[0]
    srv = gpu_lib.Server(4 * gpu_lib.server_request_bytes(r["m"], r["n"], r["k"], r["p"], q), slots=2)
    side = torch.cuda.Stream(device=A.device)
    side.wait_stream(torch.cuda.current_stream(A.device))
    with torch.cuda.stream(side):
        x = big
        for _ in range(12):  # keep the side stream busy for a few milliseconds
            x = torch.tanh(x @ big)
        A_late.copy_(A + 0.0 * x[:1, :1])  # written only after the chain
        t = srv.submit(A_late, r["k"], r["p"], q, 7, out)
    done = set()
    while t not in done:
        fin, _, _ = srv.poll()
        done.update(fin)
    srv.close()
    assert not srv.failed
    for a, b in zip(out, solo):
        assert torch.equal(a, b)


def test_budget_refuses_oversized_request(gpu_lib):
    announce("serving: oversized request")
    reqs, As = _requests(2, 4)
    r, A = reqs[0], As[0]
    srv = gpu_lib.Server(4096, slots=2)
    with pytest.raises(gpu_lib.RqlpError):
        srv.submit(A, r["k"], r["p"], 0, 1, _outs([r], A.device)[0])
    srv.close()
