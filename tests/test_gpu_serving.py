"""GPU tests of the continuous-batching scheduler (aroam_server_*): results are the same alone
and in a mix, admission respects the device-memory budget, oversized requests are rejected,
and served reduced-precision reconstructions match the FP64 oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import solvers as osol
from tests.helpers import oracle_ops, oracle_signals, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2009_10173_amd as P  # noqa: E402
from paper_2009_10173_amd import serve as S  # noqa: E402


def _small_trace(n=8, seed=5):
    tr = W.serve_trace(n, 100.0, seed, sides=(64, 96), nzs=(64,))
    # make sure both solvers and both sensors occur
    for i, r in enumerate(tr):
        r["kind"] = "lsqr" if i % 3 else "fista"
        r["sensor"] = "4mm" if i % 2 else "7mm"
    return tr


@pytest.fixture(scope="module")
def served_setup():
    assert torch.cuda.is_available()
    cache = S.ModelCache()
    reqs = S.prepare(_small_trace(), cache)
    yield cache, reqs
    cache.close()


def _run_all(reqs, mode, slots, budget, stagger=False, held=None):
    outs = []
    srv = P.aroam_server_create(budget, slots, 2)
    try:
        ids = {}
        for i, r in enumerate(reqs):
            kind, o = S.solver_opts(r["req"], mode)
            x = torch.zeros_like(r["x"])
            outs.append(x)
            ids[P.aroam_server_submit(srv, r["model"].handle, kind, r["s"], x, **o)] = i
            if stagger:
                P.aroam_server_poll(srv)
        done, max_res, status = 0, 0, {}
        while done < len(reqs):
            nres, _ = P.aroam_server_poll(srv)
            max_res = max(max_res, nres)
            for rid, info in P.aroam_server_collect(srv):
                status[ids[rid]] = info["status"]
                done += 1
        if held is not None:
            held.extend(P.aroam_server_held(srv))
    finally:
        P.aroam_server_destroy(srv)
    torch.cuda.synchronize()
    return outs, max_res, status


def test_results_equal_alone_and_in_mix(served_setup):
    _, reqs = served_setup
    budget = 64 << 30
    alone = []
    for r in reqs:
        o, _, st = _run_all([r], "bf16r", 1, budget)
        assert st[0] == 0
        alone.append(o[0])
    mix, max_res, st = _run_all(reqs, "bf16r", 8, budget, stagger=True)
    assert all(v == 0 for v in st.values())
    assert max_res > 1                      # the requests really overlapped
    for a, b in zip(alone, mix):
        assert torch.equal(a, b)


def test_served_equals_blocking_solve(served_setup):
    _, reqs = served_setup
    outs, _, st = _run_all(reqs[:3], "fp32", 4, 64 << 30)
    for r, x in zip(reqs[:3], outs):
        kind, o = S.solver_opts(r["req"], "fp32")
        ref = torch.zeros_like(r["x"])
        (P.aroam_solve_lsqr if kind == 0 else P.aroam_solve_l1)(r["model"].handle, r["s"], ref, **o)
        torch.cuda.synchronize()
        assert torch.equal(x, ref)


def test_admission_respects_budget(served_setup):
    _, reqs = served_setup
    feet = []
    for r in reqs:
        kind, o = S.solver_opts(r["req"], "bf16r")
        feet.append(P.aroam_solve_footprint(r["model"].handle, kind, **o))
    budget = int(max(feet) * 1.5)         # room for one large request at a time
    cap = int(budget // min(feet))
    held = []
    _, max_res, st = _run_all(reqs, "bf16r", 8, budget, held=held)
    assert all(v == 0 for v in st.values())
    assert 1 <= max_res <= cap
    print(f"[budget] polls held by the budget {held[0]}, by the large policy {held[1]}")
    assert held[0] >= 1 and held[1] == 0   # the budget bound while slots were free


def test_oversized_request_is_rejected(served_setup):
    _, reqs = served_setup
    r = reqs[0]
    kind, o = S.solver_opts(r["req"], "bf16r")
    foot = P.aroam_solve_footprint(r["model"].handle, kind, **o)
    _, _, st = _run_all([r], "bf16r", 2, foot // 2)
    assert st[0] == -2                    # AROAM_ENOMEM


def test_served_refined_lsqr_matches_oracle():
    name = "mid"
    cfg = W.config(name)
    m = P.Model(cfg["sensor"], cfg["grid"], dtypes=("fp32", "bf16"))
    _, s = oracle_signals(name)
    A, AT = oracle_ops(name)
    lam = osol.lam_l2(AT(s.ravel()))
    x_ref = osol.lsqr_refined(A, AT, s.ravel(), lam, 30, 2)
    st = torch.from_numpy(s.astype(np.float32)).cuda()
    x = torch.zeros(m.image_shape, device="cuda")
    srv = P.aroam_server_create(8 << 30, 4, 3)
    try:
        P.aroam_server_submit(srv, m.handle, 0, st, x, lam=-1.0, iters=30,
                              inner=P.AROAM_BF16, outer=P.AROAM_FP32, refine_sweeps=2)
        done = []
        while not done:
            P.aroam_server_poll(srv)
            done = P.aroam_server_collect(srv)
    finally:
        P.aroam_server_destroy(srv)
    assert done[0][1]["status"] == 0
    assert abs(done[0][1]["lam"] - lam) <= 1e-5 * lam
    assert rel_l2(x.cpu().numpy(), x_ref) <= 1e-4
    m.close()


def test_one_large_request_resident(served_setup):
    """With the large-request threshold between the LSQR and the FISTA requests' work, the
    FISTA requests are large: at most one is resident, the second waits at its place while
    the LSQR requests behind it are admitted, the large ones finish in submission order, and
    every result equals the request's result without the policy."""
    _, reqs = served_setup
    fista = [r for r in reqs if r["req"]["kind"] == "fista"][:2]
    lsqr = [r for r in reqs if r["req"]["kind"] == "lsqr"][:3]
    order = [fista[0], fista[1]] + lsqr
    work = [S.work_macs(r, "fp32") for r in order]
    large = max(work[2:]) * 1.01
    assert min(work[:2]) >= large            # the FISTA requests are the large ones
    ref, _, st = _run_all(order, "fp32", 8, 64 << 30)
    assert all(v == 0 for v in st.values())
    srv = P.aroam_server_create(64 << 30, 8, 2)
    try:
        P.aroam_server_set_large(srv, large)
        outs, ids = [], {}
        for i, r in enumerate(order):
            kind, o = S.solver_opts(r["req"], "fp32")
            x = torch.zeros_like(r["x"])
            outs.append(x)
            ids[P.aroam_server_submit(srv, r["model"].handle, kind, r["s"], x, **o)] = i
        with pytest.raises(P.AroamError):      # only before the first submission
            P.aroam_server_set_large(srv, large)
        nres, nq = P.aroam_server_poll(srv)
        print(f"[large policy] after the first poll: {nres} resident, {nq} queued", flush=True)
        assert (nres, nq) == (len(order) - 1, 1)   # the second FISTA request waits
        assert P.aroam_server_held(srv) == (0, 1)
        finished = []
        while len(finished) < len(order):
            P.aroam_server_poll(srv)
            for rid, info in P.aroam_server_collect(srv):
                assert info["status"] == 0
                finished.append(ids[rid])
    finally:
        P.aroam_server_destroy(srv)
    torch.cuda.synchronize()
    assert finished.index(0) < finished.index(1)
    for a, b in zip(ref, outs):
        assert torch.equal(a, b)


def test_large_request_alone(served_setup):
    """With large_alone, nothing is admitted while a large request is resident: a large
    request at the head of the queue is admitted alone, the rest waits, and results are those
    of the requests without the policy."""
    _, reqs = served_setup
    fista = [r for r in reqs if r["req"]["kind"] == "fista"][:1]
    lsqr = [r for r in reqs if r["req"]["kind"] == "lsqr"][:2]
    order = fista + lsqr
    large = max(S.work_macs(r, "fp32") for r in lsqr) * 1.01
    ref, _, _ = _run_all(order, "fp32", 8, 64 << 30)
    srv = P.aroam_server_create(64 << 30, 8, 2)
    try:
        P.aroam_server_set_large(srv, large, True)
        outs, ids = [], {}
        for i, r in enumerate(order):
            kind, o = S.solver_opts(r["req"], "fp32")
            x = torch.zeros_like(r["x"])
            outs.append(x)
            ids[P.aroam_server_submit(srv, r["model"].handle, kind, r["s"], x, **o)] = i
        assert P.aroam_server_poll(srv) == (1, 2)
        finished = []
        while len(finished) < len(order):
            P.aroam_server_poll(srv)
            for rid, info in P.aroam_server_collect(srv):
                assert info["status"] == 0
                finished.append(ids[rid])
    finally:
        P.aroam_server_destroy(srv)
    torch.cuda.synchronize()
    assert finished[0] == 0
    for a, b in zip(ref, outs):
        assert torch.equal(a, b)
