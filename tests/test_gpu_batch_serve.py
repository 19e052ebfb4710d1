"""Batched solves and the serving loop on the GPU.

* A batch of right-hand sides with different quarks (charges and kappas) on
  one field: every solution reaches a true FP64 residual <= 1e-10 (oracle D),
  and each equals, bit for bit, the solution of the same right-hand side
  solved alone -- a right-hand side's arithmetic does not depend on its
  batch-mates.
* Serving: requests on two lattices of different size, with different
  charges, kappas, sources and numbers of right-hand sides, submitted while
  others run; every result is checked against the oracle and against the
  same request solved alone.  A budget below one request's footprint still
  serves everything, one request at a time.
"""

import time

import numpy as np
import pytest

from gpu_common import Case, rel, to_dev, to_host
from oracle import dirac as od

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1710_08839_amd import qxd
    return qxd.Context(0)


@pytest.fixture(scope="module")
def big(ctx):
    return Case(ctx, (8, 8, 8, 8), cstar=3, q=2 / 3, kappa=0.13, csw=1.9, eps=0.3, seed=4)


@pytest.fixture(scope="module")
def small(ctx):
    # 4 x (2*4) x 4 x 4 C* lattice with 2^4 blocks: L1 / b1 = 2 (even)
    return Case(ctx, (4, 4, 4, 4), cstar=3, q=-1 / 3, kappa=0.128, csw=1.5, eps=0.3, seed=5,
                block=(2, 2, 2, 2))


def _ops(case, quarks):
    from oracle import fields as of
    ue, ae = of.extend_gauge(case.lat, case.u, case.a)
    return [od.build_operator(case.lat, ue, ae, k, q=q, csw=c, csw_u1=1.0) for (k, q, c) in quarks]


QUARKS = [(0.13, 2 / 3, 1.9), (0.1300, -1 / 3, 1.9), (0.126, 2 / 3, 1.2)]


@pytest.mark.parametrize("prec", [0, 1, 2, 3], ids=["f64", "f32", "f16s", "bf16"])
def test_batched_solve_matches_alone(big, prec):
    import torch
    from paper_1710_08839_amd import qxd
    c = big
    qs = [qxd.quark(k, q, cs, 1.0) for (k, q, cs) in QUARKS]
    ops = _ops(c, QUARKS)
    nsrc = 2
    etas = np.stack([c.source(700 + s) for _ in QUARKS for s in range(nsrc)])
    s = qxd.solver(kind=qxd.SAP_GCR, tol=1e-10, nkv=8, ncy=3, nmr=4, inner_prec=prec)
    psi = torch.empty_like(to_dev(etas))
    st, info = c.field.solve(qs, s, to_dev(etas), psi, nrhs=len(etas))
    assert st == 0
    ph = to_host(psi)
    for r in range(len(etas)):
        op = ops[r // nsrc]
        res = od.norm(etas[r] - op.apply(ph[r])) / od.norm(etas[r])
        assert res <= 1.05e-10, (r, res)
        assert info[r].true_resid <= 1e-10
    # each right-hand side alone gives the same bits
    for r in (0, 3, len(etas) - 1):
        one = torch.empty_like(to_dev(etas[r]))
        st1, _ = c.field.solve(qs[r // nsrc], s, to_dev(etas[r]), one)
        assert st1 == 0
        assert np.array_equal(to_host(one), ph[r]), r


def test_step_graphs_match_direct_launches(big):
    """The captured-graph replay of the batched steps gives the same bits as
    launching every kernel directly, on repeated solves (each replays the
    graph many times, with the solver's own host work and synchronisations
    in between)."""
    import torch
    from paper_1710_08839_amd import qxd
    c = big
    qs = [qxd.quark(k, q, cs, 1.0) for (k, q, cs) in QUARKS]
    etas = np.stack([c.source(800 + s) for _ in QUARKS for s in range(2)])
    s = qxd.solver(kind=qxd.SAP_GCR, tol=1e-10, nkv=8, ncy=3, nmr=4, inner_prec=qxd.F32)
    outs, counts = [], []
    try:
        for graphs in (False, True, True):
            qxd.set_step_graphs(graphs)
            c0 = qxd.step_graph_counts()
            psi = torch.empty_like(to_dev(etas))
            st, _ = c.field.solve(qs, s, to_dev(etas), psi, nrhs=len(etas))
            assert st == 0
            outs.append(to_host(psi))
            c1 = qxd.step_graph_counts()
            counts.append((c1[0] - c0[0], c1[1] - c0[1]))
    finally:
        qxd.set_step_graphs(True)
    assert counts[0] == (0, 0)
    # with graphs on, steps are launched from graphs, and some graphs again
    for cap, launches in counts[1:]:
        assert cap >= 1 and launches > cap, counts
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[0], outs[2])


def test_serve_mixed_stream(ctx, big, small):
    import torch
    from paper_1710_08839_amd import qxd, synth
    fields = {"big": big, "small": small}
    s = qxd.solver(kind=qxd.SAP_GCR, tol=1e-10, nkv=8, ncy=3, nmr=4, inner_prec=qxd.F32)
    rng = np.random.default_rng(3)
    reqs = []
    for j in range(10):
        which = "big" if j % 3 else "small"
        c = fields[which]
        k, q, cs = QUARKS[j % len(QUARKS)]
        nrhs = int(rng.integers(1, 4))
        if j % 2:
            eta = np.stack([c.source(900 + 10 * j + r) for r in range(nrhs)])
        else:
            eta = np.stack([synth.point_source(c.V, int(rng.integers(c.V)), r % 4, r % 3) for r in range(nrhs)])
        reqs.append(dict(which=which, quark=(k, q, cs), eta=eta, nrhs=nrhs))
    ctx.serve_start()
    try:
        bufs = []
        tickets = []
        for j, rq in enumerate(reqs):
            c = fields[rq["which"]]
            e = to_dev(rq["eta"])
            p = torch.empty_like(e)
            torch.cuda.synchronize()
            bufs.append((e, p))
            k, q, cs = rq["quark"]
            tickets.append(ctx.serve_submit(c.field, qxd.quark(k, q, cs, 1.0), s, e, p, rq["nrhs"]))
            if j % 4 == 3:
                time.sleep(0.05)  # later requests arrive while earlier ones run
        results = {}
        t0 = time.time()
        while len(results) < len(tickets) and time.time() - t0 < 120:
            for t in tickets:
                if t not in results:
                    r = ctx.serve_poll(t)
                    if r is not None:
                        results[t] = r
            time.sleep(0.005)
        assert len(results) == len(tickets), "serving did not finish"
    finally:
        ctx.serve_stop()
    for j, (rq, t) in enumerate(zip(reqs, tickets)):
        res = results[t]
        assert res.status == 0, (j, res.status)
        assert res.latency_s >= res.queue_s >= 0
        c = fields[rq["which"]]
        op = _ops(c, [rq["quark"]])[0]
        ph = to_host(bufs[j][1])
        for r in range(rq["nrhs"]):
            rr = od.norm(rq["eta"][r] - op.apply(ph[r])) / od.norm(rq["eta"][r])
            assert rr <= 1.05e-10, (j, r, rr)
        # the same request solved alone gives the same bits
        if j in (0, 1, 5):
            alone = torch.empty_like(bufs[j][0])
            k, q, cs = rq["quark"]
            st, _ = c.field.solve(qxd.quark(k, q, cs, 1.0), s, bufs[j][0], alone, nrhs=rq["nrhs"])
            assert st == 0
            assert np.array_equal(to_host(alone), ph), j


def test_serve_tiny_budget_serialises(ctx, small):
    import torch
    from paper_1710_08839_amd import qxd
    c = small
    s = qxd.solver(kind=qxd.SAP_GCR, tol=1e-10, nkv=6, ncy=2, nmr=3, inner_prec=qxd.F32)
    ctx.serve_start(budget_bytes=1, max_active=1)
    try:
        etas = [to_dev(c.source(50 + j)[None]) for j in range(4)]
        outs = [torch.empty_like(e) for e in etas]
        torch.cuda.synchronize()
        ts = [ctx.serve_submit(c.field, c.quark, s, e, o, 1) for e, o in zip(etas, outs)]
        done = {}
        t0 = time.time()
        while len(done) < len(ts) and time.time() - t0 < 60:
            for t in ts:
                if t not in done:
                    r = ctx.serve_poll(t)
                    if r is not None:
                        done[t] = r
            time.sleep(0.005)
    finally:
        ctx.serve_stop()
    assert len(done) == 4 and all(r.status == 0 for r in done.values())
    # one at a time: each later request waited in the queue
    qs = [done[t].queue_s for t in ts]
    assert qs[-1] > 0
    for e, o in zip(etas, outs):
        x = to_host(e)[0]
        assert od.norm(x - c.op.apply(to_host(o)[0])) / od.norm(x) <= 1.05e-10


def test_serve_errors(ctx, small):
    import torch
    from paper_1710_08839_amd import qxd
    c = small
    with pytest.raises(qxd.QxdError):
        ctx.serve_submit(c.field, c.quark, qxd.solver(), to_dev(c.source(1)), torch.empty(1, device="cuda"), 1)
    ctx.serve_start()
    try:
        with pytest.raises(qxd.QxdError):  # EO_GCR is not served
            e = to_dev(c.source(1))
            ctx.serve_submit(c.field, c.quark, qxd.solver(kind=qxd.EO_GCR), e, torch.empty_like(e), 1)
        with pytest.raises(qxd.QxdError):
            ctx.serve_poll(123456)
    finally:
        ctx.serve_stop()


def test_operator_cache_eviction(ctx, small):
    """More distinct operators than a field keeps cached: every application
    matches the oracle, an operator rebuilt after eviction gives the same bits,
    and a batched solve holding more operators than the cache keeps (all in
    use, none evictable) converges for every right-hand side."""
    import torch
    from paper_1710_08839_amd import qxd
    c = small
    x = c.source(900)
    kappas = [0.120 + 0.001 * i for i in range(7)]
    quarks = [(k, -1 / 3, 1.5) for k in kappas]
    ops = _ops(c, quarks)
    first = None
    for (k, q, cs), op in zip(quarks, ops):
        y = torch.empty_like(to_dev(x))
        c.field.apply(qxd.quark(k, q, cs, 1.0), qxd.OP_D, 0, to_dev(x), y)
        torch.cuda.synchronize()
        assert rel(to_host(y), op.apply(x)) < 1e-12, k
        if first is None:
            first = to_host(y)
    y = torch.empty_like(to_dev(x))
    c.field.apply(qxd.quark(*quarks[0], 1.0), qxd.OP_D, 0, to_dev(x), y)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(y), first)
    qs = [qxd.quark(k, q, cs, 1.0) for (k, q, cs) in quarks[:6]]
    etas = np.stack([c.source(910 + r) for r in range(6)])
    s = qxd.solver(kind=qxd.SAP_GCR, tol=1e-10, nkv=8, ncy=3, nmr=4, inner_prec=qxd.F32)
    psi = torch.empty_like(to_dev(etas))
    st, info = c.field.solve(qs, s, to_dev(etas), psi, nrhs=6)
    assert st == 0
    ph = to_host(psi)
    for r in range(6):
        assert od.norm(etas[r] - ops[r].apply(ph[r])) / od.norm(etas[r]) <= 1.05e-10, r


def test_failed_step_ends_solves_and_requests(ctx, small):
    """A batched step that fails (forced from the host before any launch)
    ends every right-hand side in flight with the error: qxd_solve returns it
    with each info.status set, a served request completes with it, and the
    serve loop still stops.  Afterwards the same solve succeeds."""
    import torch
    from paper_1710_08839_amd import qxd
    c = small
    s = qxd.solver(kind=qxd.SAP_GCR, tol=1e-10, nkv=6, ncy=2, nmr=3, inner_prec=qxd.F32)
    etas = to_dev(np.stack([c.source(60 + r) for r in range(3)]))
    psi = torch.empty_like(etas)
    qxd.fail_steps(1)
    try:
        st, info = c.field.solve(c.quark, s, etas, psi, nrhs=3, check=False)
    finally:
        qxd.fail_steps(0)
    assert st == -5 and all(i.status == -5 for i in info)
    ctx.serve_start()
    try:
        qxd.fail_steps(1)
        t = ctx.serve_submit(c.field, c.quark, s, etas, psi, 3)
        r, t0 = None, time.time()
        while r is None and time.time() - t0 < 30:
            r = ctx.serve_poll(t)
            time.sleep(0.005)
    finally:
        qxd.fail_steps(0)
        ctx.serve_stop()
    assert r is not None and r.status == -5
    st, info = c.field.solve(c.quark, s, etas, psi, nrhs=3)
    assert st == 0
    ph, eh = to_host(psi), to_host(etas)
    for k in range(3):
        assert od.norm(eh[k] - c.op.apply(ph[k])) / od.norm(eh[k]) <= 1.05e-10


def test_serve_charges_drain(ctx, small):
    """Requests with distinct quarks (each builds its own operator) all
    complete; while they run the operators being built are charged, and once
    they are done nothing stays charged as pending, the operators left are
    the field's bounded cache (at most four unused ones), and the groups give
    their solver slots back when idle."""
    import torch
    from paper_1710_08839_amd import qxd
    c = small
    s = qxd.solver(kind=qxd.SAP_GCR, tol=1e-10, nkv=6, ncy=2, nmr=3, inner_prec=qxd.F32)
    kappas = [0.1205 + 0.0007 * j for j in range(8)]
    etas = [to_dev(c.source(700 + j)[None]) for j in range(len(kappas))]
    outs = [torch.empty_like(e) for e in etas]
    torch.cuda.synchronize()
    ctx.serve_start()
    try:
        ts = [ctx.serve_submit(c.field, qxd.quark(k, -1 / 3, 1.5, 1.0), s, e, o, 1)
              for k, e, o in zip(kappas, etas, outs)]
        done, t0 = {}, time.time()
        while len(done) < len(ts) and time.time() - t0 < 60:
            for t in ts:
                if t not in done:
                    r = ctx.serve_poll(t)
                    if r is not None:
                        done[t] = r
            time.sleep(0.005)
        ch = ctx.serve_charges()
        t0 = time.time()
        while ch["slots"] and time.time() - t0 < 10:
            time.sleep(0.02)
            ch = ctx.serve_charges()
    finally:
        ctx.serve_stop()
    assert len(done) == len(ts) and all(r.status == 0 for r in done.values())
    assert ch["op_pending"] == 0 and ch["slots"] == 0
    one_op = 36 * (2 * c.V + c.V // 2) * (16 + 8)  # Pauli term, inverse, links: FP64 and FP32
    assert ch["op_resident"] <= 4 * one_op
    ops = _ops(c, [(k, -1 / 3, 1.5) for k in kappas])
    for e, o, op in zip(etas, outs, ops):
        x = to_host(e)[0]
        assert od.norm(x - op.apply(to_host(o)[0])) / od.norm(x) <= 1.05e-10


def test_serve_admits_requests_in_pieces(ctx, small):
    """With a budget that holds no solver slot at all, a request of three
    right-hand sides is admitted one right-hand side at a time (each when no
    other work is charged) and completes with every solution correct; the
    request behind it waits until all three are in."""
    import torch
    from paper_1710_08839_amd import qxd
    c = small
    s = qxd.solver(kind=qxd.SAP_GCR, tol=1e-10, nkv=6, ncy=2, nmr=3, inner_prec=qxd.F32)
    e3 = to_dev(np.stack([c.source(80 + j) for j in range(3)]))
    e1 = to_dev(c.source(90)[None])
    o3, o1 = torch.empty_like(e3), torch.empty_like(e1)
    torch.cuda.synchronize()
    ctx.serve_start(budget_bytes=1)
    try:
        t3 = ctx.serve_submit(c.field, c.quark, s, e3, o3, 3)
        t1 = ctx.serve_submit(c.field, c.quark, s, e1, o1, 1)
        done, t0 = {}, time.time()
        while len(done) < 2 and time.time() - t0 < 60:
            for t in (t3, t1):
                if t not in done:
                    r = ctx.serve_poll(t)
                    if r is not None:
                        done[t] = r
            time.sleep(0.005)
    finally:
        ctx.serve_stop()
    assert len(done) == 2 and done[t3].status == 0 and done[t1].status == 0
    assert done[t3].nrhs == 3
    # the second request was admitted only after the first one's last piece
    assert done[t1].queue_s > 0
    eh, oh = to_host(e3), to_host(o3)
    for j in range(3):
        assert od.norm(eh[j] - c.op.apply(oh[j])) / od.norm(eh[j]) <= 1.05e-10, j
    x = to_host(e1)[0]
    assert od.norm(x - c.op.apply(to_host(o1)[0])) / od.norm(x) <= 1.05e-10
