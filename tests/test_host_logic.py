"""Host logic without a GPU: the serving loop driven by a fake executor (the server's admission
rule over simulated requests: budget, max_active, option groups, ticket order) and the
training driver's learning-rate schedule."""
import numpy as np
import pytest

import paper_2402_08296_amd as dg

OK, E_BUDGET, E_INVALID = 0, -8, -1
C = 0.01  # seconds per chunk


def req(arrival=0.0, setup_s=0.0, bytes=10, group=1, chunks=1, setup_ok=1):
    return dict(arrival=arrival, setup_s=setup_s, bytes=bytes, group=group, chunks=chunks, setup_ok=setup_ok)


def test_unbounded_server_runs_everything_at_once():
    out = dg.simulate_server([req(chunks=k) for k in (3, 1, 5, 2)], hbm_budget=1 << 40, max_active=64, chunk_s=C)
    for (adm, fin, st), k in zip(out, (3, 1, 5, 2)):
        assert st == OK and adm == 0.0
        assert fin == pytest.approx(k * C)


def test_budget_serializes_and_oversized_is_rejected():
    rs = [req(bytes=60, chunks=2), req(bytes=60, chunks=2), req(bytes=101), req(bytes=40, chunks=1)]
    out = dg.simulate_server(rs, hbm_budget=100, max_active=8, chunk_s=C)
    assert out[2] == (0.0, 0.0, E_BUDGET)
    assert out[0][0] == 0.0 and out[0][1] == pytest.approx(2 * C)
    # the second does not fit beside the first; the fourth would fit (60 + 40) but may not overtake it
    assert out[1][0] == pytest.approx(2 * C) and out[1][1] == pytest.approx(4 * C)
    assert out[3][0] == pytest.approx(2 * C) and out[3][1] == pytest.approx(3 * C)


def test_max_active():
    out = dg.simulate_server([req(chunks=1) for _ in range(5)], hbm_budget=1 << 40, max_active=2, chunk_s=C)
    adm = [o[0] for o in out]
    assert adm == pytest.approx([0, 0, C, C, 2 * C])


def test_group_drains_before_another_and_no_overtaking():
    rs = [req(group=1, chunks=3), req(group=2, chunks=1), req(group=1, chunks=1)]
    out = dg.simulate_server(rs, hbm_budget=1 << 40, max_active=8, chunk_s=C)
    # the group-2 request waits for group 1 to drain; the later group-1 request waits behind it
    assert out[0][:2] == pytest.approx((0, 3 * C))
    assert out[1][:2] == pytest.approx((3 * C, 4 * C))
    assert out[2][:2] == pytest.approx((4 * C, 5 * C))


def test_setup_workers_and_failed_setup():
    rs = [req(setup_s=1.0), req(setup_s=1.0, setup_ok=0), req(setup_s=1.0), req(arrival=5.0, setup_s=0.5)]
    out = dg.simulate_server(rs, hbm_budget=1 << 40, max_active=8, setup_threads=1, chunk_s=C)
    assert out[0][0] == pytest.approx(1.0)
    assert out[1][2] == E_INVALID and out[1][0] == pytest.approx(2.0)
    assert out[2][0] == pytest.approx(3.0)
    assert out[3][0] == pytest.approx(5.5)  # idle server waits for the next setup
    out4 = dg.simulate_server(rs[:3], hbm_budget=1 << 40, max_active=8, setup_threads=4, chunk_s=C)
    assert [o[0] for o in out4] == pytest.approx([1.0, 1.0, 1.0])


def test_invalid_arguments():
    with pytest.raises(dg.DDMGNNError):
        dg.simulate_server([req()], hbm_budget=0, max_active=1)
    with pytest.raises(dg.DDMGNNError):
        dg.simulate_server([req(arrival=1.0), req(arrival=0.5)], hbm_budget=100, max_active=1)
    with pytest.raises(dg.DDMGNNError):
        dg.simulate_server([req(chunks=0)], hbm_budget=100, max_active=1)
    assert dg.simulate_server([], hbm_budget=100, max_active=1) == []


@pytest.mark.parametrize("seed", range(6))
def test_random_streams_keep_the_invariants(seed):
    """Poisson arrivals, mixed sizes, groups and lengths: every admitted set fits the
    budget and max_active and shares one group, a request runs exactly its chunks,
    no ready request is passed by a later one, and p50/p99 latency are ordered."""
    g = np.random.default_rng(seed)
    n, budget, max_active = 300, 1000, 6
    t = np.cumsum(g.exponential(0.02, n))
    rs = [req(arrival=float(t[i]), setup_s=float(g.uniform(0.0, 0.05)), bytes=int(g.integers(50, 1100)),
              group=int(g.integers(1, 3)), chunks=int(g.integers(1, 8))) for i in range(n)]
    out = dg.simulate_server(rs, hbm_budget=budget, max_active=max_active, setup_threads=3, chunk_s=C)
    ok = [i for i in range(n) if out[i][2] == OK]
    for i in range(n):
        if rs[i]["bytes"] > budget:
            assert out[i][2] == E_BUDGET
        else:
            assert out[i][2] == OK
    events = sorted({out[i][0] for i in ok})
    for te in events:
        live = [i for i in ok if out[i][0] <= te + 1e-12 and out[i][1] > te + 1e-12]
        assert sum(rs[i]["bytes"] for i in live) <= budget
        assert len(live) <= max_active
        assert len({rs[i]["group"] for i in live}) <= 1
    for i in ok:
        assert out[i][1] - out[i][0] == pytest.approx(rs[i]["chunks"] * C)
        assert out[i][0] >= rs[i]["arrival"] + rs[i]["setup_s"] - 1e-12
    # setup order: one finished setup before j's admission is admitted no later than j
    ready = {}
    free = [0.0] * 3
    for i in range(n):
        w = int(np.argmin(free))
        free[w] = max(free[w], rs[i]["arrival"]) + rs[i]["setup_s"]
        ready[i] = free[w]
    for a in range(len(ok)):
        for b in range(a + 1, len(ok)):
            i, j = ok[a], ok[b]
            if ready[i] <= out[j][0] - 1e-12:
                assert out[i][0] <= out[j][0] + 1e-12
    lat = np.array([out[i][1] - rs[i]["arrival"] for i in ok])
    p50, p99 = np.percentile(lat, [50, 99])
    assert 0 < p50 <= p99 <= lat.max()


def test_training_plateau_schedule():
    """Host logic of the training driver: the learning rate drops by the factor after more
    than `patience` epochs without a new best loss, and the count restarts."""
    from paper_2402_08296_amd import train as T
    st = T.TrainState(None, None, None, None, lr=1e-2)
    for loss in [5.0, 4.0, 4.5, 4.2, 4.1]:
        T.plateau(st, loss, patience=2, factor=0.1)
    assert st.lr == pytest.approx(1e-3) and st.best == 4.0 and st.stale == 0
    T.plateau(st, 3.0, patience=2)
    assert st.best == 3.0 and st.lr == pytest.approx(1e-3)
    assert st.history == [5.0, 4.0, 4.5, 4.2, 4.1, 3.0]
