"""Request engine on the GPU: results are the same alone and in a concurrent
mix (bitwise), applies against resident factors, failure propagation."""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import operators as ops

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bf():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2002_03400_amd as m
    m.lib()
    return m


def _t(x):
    import torch
    return torch.from_numpy(np.asarray(x, np.complex64)).cuda()


def test_max_constructs_runs_constructions_one_at_a_time(bf):
    """bf_server_opts.max_constructs = 1 on 4 slots: the queued constructions
    run one after another (each starts once the previous one has finished),
    an apply against a finished construction still takes an idle slot beside
    them, and the factors are bitwise those of each construction alone."""
    import torch
    specs = [(2048, 8.0, 1e-6, 21), (3000, 8.0, 1e-6, 22), (2500, 6.0, 1e-6, 23)]
    opsl = []
    for n, ppw, tol, seed in specs:
        g = wl.segment_pair(n, ppw=ppw)
        opsl.append(bf.segkernel(g.targets, g.sources, g.k))
    say("alone")
    alone = []
    for op, (n, ppw, tol, seed) in zip(opsl, specs):
        F = bf.construct(op, tol, 64, seed=seed)
        alone.append(F.export())
        F.close()
    say("capped server")
    S = bf.Server(slots=4, max_constructs=1)
    t0 = S.submit_construct(opsl[0], specs[0][2], 64, seed=specs[0][3])
    S.wait(t0)
    rest = [S.submit_construct(op, tol, 64, seed=seed)
            for op, (n, ppw, tol, seed) in zip(opsl[1:], specs[1:])]
    ta = S.submit_apply(t0, _t(np.ones((specs[0][0], 1))))
    infos = [S.wait(t) for t in rest]
    ia = S.wait(ta)
    torch.cuda.synchronize()
    first, second = sorted(infos, key=lambda i: i["start_ns"])
    say("constructions", first["start_ns"], first["finish_ns"], second["start_ns"],
        "apply", ia["start_ns"])
    assert second["start_ns"] >= first["finish_ns"]
    assert ia["start_ns"] < second["finish_ns"]
    for t, a in zip([t0] + rest, alone):
        assert np.array_equal(S.factors(t).export(), a)
    S.close()
    with pytest.raises(bf.BFError):
        bf.Server(slots=2, max_constructs=-1)


@pytest.mark.parametrize("rounds", [False, True])
def test_mix_equals_alone(bf, rounds):
    """Constructions of several sizes, wavenumbers and tolerances run together
    on 4 slots give bitwise the factors each gives alone, with and without
    cross-request solve rounds (their QRs and least squares then share
    persistent launches)."""
    import torch
    specs = [(2048, 8.0, 1e-6, 11), (3000, 4.0, 1e-4, 12), (4096, 16.0, 1e-6, 13),
             (2500, 6.0, 1e-6, 14), (5000, 8.0, 1e-4, 15), (2048, 12.0, 1e-4, 16)]
    opsl = []
    for n, ppw, tol, seed in specs:
        g = wl.segment_pair(n, ppw=ppw)
        opsl.append(bf.segkernel(g.targets, g.sources, g.k))
    say("alone")
    alone = []
    for op, (n, ppw, tol, seed) in zip(opsl, specs):
        F = bf.construct(op, tol, 64, seed=seed)
        alone.append(F.export())
        F.close()
    say("mix", "rounds" if rounds else "")
    S = bf.Server(slots=4, solve_rounds=rounds)
    tickets = [S.submit_construct(op, tol, 64, seed=seed) for op, (n, ppw, tol, seed) in zip(opsl, specs)]
    for t, a in zip(tickets, alone):
        info = S.wait(t)
        assert info["finish_ns"] >= info["start_ns"] >= info["arrival_ns"]
        got = S.factors(t).export()
        assert np.array_equal(got, a)
    nr, ni = S.rounds()
    say("solve rounds", nr, "items", ni)
    if rounds:
        # the QRs of every leaf-loop pass and sweep level and the centre
        # least squares of every construction went through rounds
        assert nr > 0 and ni > 0
    else:
        assert (nr, ni) == (0, 0)
    # applies against resident factors, from several requests at once
    X = [_t(wl.test_columns(n, 3, 5)) for (n, _, _, _) in specs]
    at = [S.submit_apply(t, x) for t, x in zip(tickets, X)]
    for k, (t, a_t) in enumerate(zip(tickets, at)):
        S.wait(a_t)
        ref = S.factors(t).apply(X[k])
        torch.cuda.synchronize()
        assert torch.equal(S.result(a_t), ref)
    S.close()


def test_failed_construction_fails_its_applies(bf):
    g = wl.segment_pair(512, ppw=8.0)
    op = bf.segkernel(g.targets, g.sources, g.k)
    S = bf.Server(slots=2)
    t = S.submit_construct(op, 1e-6, 64, seed=1, max_rank=2)     # rank cap -> BF_ERANK
    a = S.submit_apply(t, _t(np.ones((512, 1))))
    with pytest.raises(bf.BFError) as e1:
        S.wait(t)
    assert e1.value.code == -4
    with pytest.raises(bf.BFError):
        S.wait(a)
    S.close()


def test_budget_serializes_but_completes(bf):
    """A budget smaller than one request still runs every request (alone)."""
    g = wl.segment_pair(1024, ppw=8.0)
    op = bf.segkernel(g.targets, g.sources, g.k)
    S = bf.Server(slots=3, hbm_budget=1 << 20)
    ts = [S.submit_construct(op, 1e-6, 32, seed=s) for s in range(4)]
    spans = []
    for t in ts:
        i = S.wait(t)
        spans.append((i["start_ns"], i["finish_ns"]))
    spans.sort()
    for (s0, f0), (s1, f1) in zip(spans, spans[1:]):
        assert s1 >= f0          # never two in flight under this budget
    S.close()


@pytest.mark.parametrize("trans", [False, True])
def test_continuous_batching_of_applies(bf, trans):
    """Applies queued behind their construction are merged into one product
    (batch_cols = 64): each result matches its lone apply to single precision,
    requests are merged (batch > 1), the column cap is respected, and applies
    against another factorization are not mixed in."""
    n = 3000
    g = wl.segment_pair(n, ppw=8.0)
    op = bf.segkernel(g.targets, g.sources, g.k)
    g2 = wl.segment_pair(n, ppw=6.0)
    op2 = bf.segkernel(g2.targets, g2.sources, g2.k)
    S = bf.Server(slots=2, batch_cols=64)
    t1 = S.submit_construct(op, 1e-6, 32, seed=3)
    t2 = S.submit_construct(op2, 1e-6, 32, seed=4)
    rng = np.random.default_rng(6)
    widths = [1, 3, 5, 1, 16, 2, 30, 4, 1, 7]
    reqs = []
    for q, w in enumerate(widths):
        X = (rng.standard_normal((n, w)) + 1j * rng.standard_normal((n, w))).astype(np.complex64)
        target = t1 if q % 3 else t2
        reqs.append((target, X, S.submit_apply(target, _t(X), trans=trans)))
    infos = [S.wait(t) for _, _, t in reqs]
    say("batch sizes", [i["batch"] for i in infos])
    assert max(i["batch"] for i in infos) > 1
    F1, F2 = S.factors(t1), S.factors(t2)
    for (target, X, t), info in zip(reqs, infos):
        F = F1 if target == t1 else F2
        lone = F.apply(_t(X), trans=trans).cpu().numpy()
        got = S.result(t).cpu().numpy()
        assert np.linalg.norm(got - lone) <= 1e-6 * np.linalg.norm(lone), (t, info["batch"])
    # merged products stay within the column cap and within one factorization
    starts = {}
    for (target, X, t), info in zip(reqs, infos):
        starts.setdefault((info["start_ns"], target), []).append(X.shape[1])
    for (_, target), cols in starts.items():
        assert sum(cols) <= 64
    S.close()
