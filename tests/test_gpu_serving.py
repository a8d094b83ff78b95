"""GPU tests of the serving loop (bsim_server_*): every result is the same
alone and in a mix of overlapping requests (and equals the oracle), updates
of one state keep their order, and admission respects the memory budget."""

import numpy as np
import pytest

from oracle import oracle as orc
from oracle.updates import apply_ops
from paper_2111_12493_amd import binding
from paper_2111_12493_amd import graphgen as gg

from gpu_util import assert_same

pytestmark = pytest.mark.gpu
UNB = binding.K_UNBOUNDED


def fetch(res):
    d = res.to_dict()
    res.free()
    return d


def make_requests(seed):
    rng = np.random.default_rng(seed)
    graphs = [gg.rmat_graph(int(rng.integers(8, 13)), int(rng.integers(1000, 40000)), n_types=16, n_labels=8,
                            seed=int(rng.integers(1, 1 << 30))) for _ in range(12)]
    graphs.append(gg.append_chains(gg.uniform_graph(500, 2000, 4, 4, seed=3), 2, 150, type_id=4))
    base = gg.uniform_graph(3000, 15000, 8, 8, seed=9)
    batches, g = [], base
    for i in range(6):
        d = gg.update_ops(g, rng, int(rng.integers(1, 400)), n_labels=8, n_types=8)
        ops = gg.ops_as_tuples(d)
        g = apply_ops(g, ops)
        batches.append((ops, g))
    return graphs, base, batches


def run(graphs, base, batches, workers, one_at_a_time):
    srv = binding.Server(workers=workers)
    out = {}
    try:
        t = srv.submit_summarize(binding.HostGraph(base), k_max=4, stop_at_fixpoint=False, keep_state=True)
        res, state = srv.poll(t)
        out["base"] = fetch(res)
        tickets = []
        order = []  # summaries and updates interleaved
        for i in range(max(len(graphs), len(batches))):
            if i < len(graphs):
                order.append(("g", i))
            if i < len(batches):
                order.append(("u", i))
        keep = []
        for kind, i in order:
            if kind == "g":
                tk = srv.submit_summarize(binding.HostGraph(graphs[i]), k_max=UNB)
            else:
                b = binding.UpdateBatch(batches[i][0])
                keep.append(b)
                tk = srv.submit_update(state, b)
            tickets.append(((kind, i), tk))
            if one_at_a_time:
                out[(kind, i)] = fetch(srv.poll(tk)[0])
        for key, tk in tickets:
            if key not in out:
                out[key] = fetch(srv.poll(tk)[0])
        st = srv.stats()
        assert st["completed"] == st["submitted"] == len(order) + 1 and st["failed"] == 0
        srv.release_state(state)
        assert srv.stats()["bytes_in_use"] == 0
    finally:
        srv.free()
    return out


def test_same_alone_and_in_the_mix():
    graphs, base, batches = make_requests(61)
    alone = run(graphs, base, batches, workers=1, one_at_a_time=True)
    mixed = run(graphs, base, batches, workers=6, one_at_a_time=False)
    assert set(alone) == set(mixed)
    for key in alone:
        assert_same(mixed[key], alone[key], key)
    # and both equal the oracle
    for i, g in enumerate(graphs):
        assert_same(alone[("g", i)], orc.summarize(g, g.n + 2, True), ("g", i))
    assert_same(alone["base"], orc.summarize(base, 4, False), "base")
    for i, (_, g) in enumerate(batches):
        assert_same(alone[("u", i)], orc.summarize(g, 4, False), ("u", i))


def test_admission_by_footprint():
    g = gg.uniform_graph(2000, 10000, 4, 4, seed=5)
    srv = binding.Server(mem_budget=4 << 20, workers=4)
    try:
        big = gg.uniform_graph(200000, 1000000, 4, 4, seed=6)
        with pytest.raises(binding.BsimError) as e:
            srv.submit_summarize(binding.HostGraph(big))
        assert e.value.status == binding.E_BUSY
        # each request fits the budget alone but not several at once: they queue
        ts = [srv.submit_summarize(binding.HostGraph(g), k_max=6) for _ in range(6)]
        ref = orc.summarize(g, 6, True)
        for t in ts:
            assert_same(fetch(srv.poll(t)[0]), ref, "queued")
        assert srv.stats()["bytes_in_use"] == 0
    finally:
        srv.free()


def test_failed_request_reports_its_error():
    srv = binding.Server(workers=2)
    try:
        good = gg.chain(3)
        bad = gg.Graph(**{**good.__dict__, "alive": np.array([1, 1, 0, 1], dtype=np.uint8)})
        t1 = srv.submit_summarize(binding.HostGraph(bad))
        t2 = srv.submit_summarize(binding.HostGraph(good))
        with pytest.raises(binding.BsimError) as e:
            srv.poll(t1)
        assert e.value.status == binding.E_INVALID
        assert_same(fetch(srv.poll(t2)[0]), orc.summarize(good, good.n + 2, True))
    finally:
        srv.free()


def test_direction_requests_in_the_mix():
    # summarize requests with the direction parameterization, served together,
    # each equal to the oracle; a state cannot take a direction flag
    rng = np.random.default_rng(61)
    graphs = [gg.rmat_graph(int(rng.integers(8, 12)), int(rng.integers(1000, 20000)), n_types=8, n_labels=6,
                            seed=int(rng.integers(1, 1 << 30))) for _ in range(9)]
    dirs = ["in", "both", "out"] * 3
    srv = binding.Server(workers=4)
    try:
        tickets = [srv.submit_summarize(binding.HostGraph(g), k_max=UNB, direction=d) for g, d in zip(graphs, dirs)]
        for g, d, t in zip(graphs, dirs, tickets):
            got = fetch(srv.poll(t)[0])
            assert_same(got, orc.summarize_ext(g, g.n + 2, True, False, d), ("serving", d))
        with pytest.raises(binding.BsimError):
            srv.submit_summarize(binding.HostGraph(graphs[0]), k_max=3, stop_at_fixpoint=False, keep_state=True,
                                 direction="in")
    finally:
        srv.free()


def test_previous_level_edge_requests():
    # summarize requests with BSIM_PREV_LEVEL_EDGES at a cap, served
    # together with plain ones, each equal to the oracle; a state refuses it
    rng = np.random.default_rng(62)
    graphs = [gg.rmat_graph(int(rng.integers(8, 12)), int(rng.integers(1000, 20000)), n_types=8, n_labels=6,
                            seed=int(rng.integers(1, 1 << 30))) for _ in range(6)]
    prev = [True, False] * 3
    srv = binding.Server(workers=4)
    try:
        tickets = [srv.submit_summarize(binding.HostGraph(g), k_max=3, stop_at_fixpoint=False, prev_level_edges=p)
                   for g, p in zip(graphs, prev)]
        for g, p, t in zip(graphs, prev, tickets):
            got = fetch(srv.poll(t)[0])
            assert_same(got, orc.summarize(g, 3, False, False, prev_level_edges=p), ("serving prev", p))
        with pytest.raises(binding.BsimError) as e:
            srv.submit_summarize(binding.HostGraph(graphs[0]), k_max=3, stop_at_fixpoint=False, keep_state=True,
                                 prev_level_edges=True)
        assert e.value.status == binding.E_UNSUPPORTED
    finally:
        srv.free()


def test_update_that_cannot_fit_beside_owned_states_is_refused():
    # a server-owned state stays in the budget; an update needs a quarter of
    # the state on top, so under a budget the state nearly fills it is refused
    # at submit (BSIM_E_BUSY) instead of queueing for good
    g = gg.uniform_graph(3000, 15000, 8, 8, seed=9)
    budget = 80 << 20
    srv = binding.Server(mem_budget=budget, workers=2)
    try:
        res, state = srv.poll(srv.submit_summarize(binding.HostGraph(g), k_max=3, stop_at_fixpoint=False,
                                                   keep_state=True))
        res.free()
        owned = srv.stats()["bytes_in_use"]
        assert owned + owned // 4 + (1 << 20) > budget, owned
        d = gg.update_ops(g, np.random.default_rng(3), 50, n_labels=8, n_types=8)
        batch = binding.UpdateBatch(gg.ops_as_tuples(d))
        with pytest.raises(binding.BsimError) as e:
            srv.submit_update(state, batch)
        assert e.value.status == binding.E_BUSY
        # small summaries still fit beside the state and run
        t = srv.submit_summarize(binding.HostGraph(gg.chain(5)))
        got = fetch(srv.poll(t)[0])
        assert_same(got, orc.summarize(gg.chain(5), 7, True), "beside the state")
        # a ticket is collected once; polling it again fails at once
        with pytest.raises(binding.BsimError) as e:
            srv.poll(t)
        assert e.value.status == binding.E_INVALID
        srv.release_state(state)
        assert srv.stats()["bytes_in_use"] == 0
    finally:
        srv.free()


def test_free_cancels_queued_requests():
    # one worker, a queue of requests: free returns (the running request
    # finishes, the queued ones are cancelled) instead of waiting for all
    g = gg.uniform_graph(20000, 100000, 4, 4, seed=5)
    srv = binding.Server(workers=1)
    for _ in range(8):
        srv.submit_summarize(binding.HostGraph(g), k_max=UNB)
    srv.free()
