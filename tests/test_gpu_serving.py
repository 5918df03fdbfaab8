"""The request server (rqlp_server_*): requests admitted while others run,
under an HBM budget that forces queueing, each give bitwise the result of the
same request run alone."""
import numpy as np
import pytest
import torch

import workloads
from tests.gpu_util import announce, to_dev

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
    for t, i in tickets.items():
        for a, b in zip(outs[i], solo[i]):
            assert torch.equal(a, b), f"request {i} differs from its solo run"


def test_budget_refuses_oversized_request(gpu_lib):
    announce("serving: oversized request")
    reqs, As = _requests(2, 4)
    r, A = reqs[0], As[0]
    srv = gpu_lib.Server(4096, slots=2)
    with pytest.raises(gpu_lib.RqlpError):
        srv.submit(A, r["k"], r["p"], 0, 1, _outs([r], A.device)[0])
    srv.close()
