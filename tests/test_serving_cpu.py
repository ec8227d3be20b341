"""Serving scheduler on the CPU with a fake backend: admission by HBM budget,
continuous batching, failure handling, latency accounting."""
from paper_2504_05148_amd.serving import FakeBackend, Server, poisson_arrivals, summarize


def test_budget_bounds_slots_and_everything_completes():
    be = FakeBackend(cost=[0.002, 0.004], slot_bytes=[10, 30])
    srv = Server(be, 2, hbm_budget=50, max_batch=4)
    arr = poisson_arrivals([400.0, 300.0], 0.3, pool_size=4, seed=1)
    fin = srv.run(arr, realtime=True)
    assert len(fin) == len(arr) and not srv.failed
    assert srv.peak_bytes <= 50
    assert all(r.done >= r.start >= r.arrival for r in fin)


def test_continuous_batching_under_load():
    # one slot, one stream: requests arriving during a launch join the next one
    be = FakeBackend(cost=[0.01], slot_bytes=[1])
    srv = Server(be, 1, hbm_budget=1, max_batch=4, n_streams=1)
    arr = [(0.001 * i, 0, i % 3) for i in range(40)]
    fin = srv.run(arr, realtime=True)
    assert len(fin) == 40
    assert max(srv.batches) == 4 and sum(k * v for k, v in srv.batches.items()) == 40
    # every launch after the first takes what queued while the previous ran
    assert srv.batches[4] >= 8


def test_rig_larger_than_budget_is_rejected_others_complete():
    # one slot of rig 1 exceeds the whole budget: its requests fail at
    # admission instead of waiting forever, rig 0 is served, run() returns
    be = FakeBackend(cost=[0.001, 0.001], slot_bytes=[10, 100])
    srv = Server(be, 2, hbm_budget=50, max_batch=2)
    arr = [(0.0, 0, 0), (0.0, 1, 0), (0.001, 0, 1), (0.002, 1, 1)]
    fin = srv.run(arr, realtime=True)
    assert sorted(r.rig for r in fin) == [0, 0]
    assert sorted(r.rig for r in srv.failed) == [1, 1]
    assert 1 in srv.rejected and "budget" in srv.rejected[1]
    # rig 0 may hold one or two slots (the second request can arrive while
    # the first launch still runs); a rig-1 slot would exceed the budget
    assert srv.peak_bytes in (10, 20) and not srv.slots[1]


def test_rig_with_invalid_parameters_is_rejected_others_unaffected():
    be = FakeBackend(cost=[0.001, 0.001, 0.001], slot_bytes=[1, 1, 1], bad_rigs=[1])
    srv = Server(be, 3, hbm_budget=10, max_batch=2)
    arr = poisson_arrivals([400.0, 400.0, 400.0], 0.05, pool_size=2, seed=4)
    fin = srv.run(arr, realtime=True)
    n1 = sum(1 for a in arr if a[1] == 1)
    assert len(srv.failed) == n1 and all(r.rig == 1 for r in srv.failed)
    assert len(fin) == len(arr) - n1 and {r.rig for r in fin} == {0, 2}
    assert "parameters rejected" in srv.rejected[1] and not srv.slots[1]


def test_rig_without_slot_takes_an_idle_slot_of_another_rig():
    # budget for two slots: rig 0 fills both with overlapping launches, then
    # goes quiet; rig 1 arrives later and must get room by releasing one of
    # rig 0's idle slots (no livelock)
    be = FakeBackend(cost=[0.02, 0.001], slot_bytes=[5, 5])
    srv = Server(be, 2, hbm_budget=10, max_batch=1)
    arr = [(0.0, 0, 0), (0.0001, 0, 1), (0.05, 1, 0), (0.051, 1, 1)]
    fin = srv.run(arr, realtime=True)
    assert len(fin) == 4 and not srv.failed
    assert srv.released[0] >= 1 and srv.peak_bytes <= 10
    assert [r.rig for r in sorted(fin, key=lambda r: r.start)] == [0, 0, 1, 1]


def test_silent_rig_releases_its_state_after_timeout():
    be = FakeBackend(cost=[0.001, 0.001], slot_bytes=[1, 1])
    srv = Server(be, 2, hbm_budget=10, max_batch=2, idle_timeout=0.05)
    srv.preallocate(2)
    # rig 1 sends two frames early and stops; rig 0 keeps sending for 0.3 s
    arr = sorted([(0.001, 1, 0), (0.002, 1, 1)] +
                 [(0.01 * i, 0, i % 2) for i in range(30)])
    fin = srv.run(arr, realtime=True)
    assert len(fin) == len(arr) and not srv.failed
    assert not srv.slots[1] and srv.released[1] == 2      # rig 1's state released
    assert srv.slots[0] and srv.released[0] == 0          # rig 0 kept its slots
    assert be.live == len(srv.slots[0])


def test_failed_launches_release_resources():
    be = FakeBackend(cost=[0.001, 0.001], slot_bytes=[1, 1], fail_rigs=[1])
    srv = Server(be, 2, hbm_budget=10, max_batch=2)
    arr = poisson_arrivals([500.0, 500.0], 0.05, pool_size=2, seed=3)
    fin = srv.run(arr, realtime=True)
    n1 = sum(1 for a in arr if a[1] == 1)
    assert len(srv.failed) == n1 and all(r.rig == 1 for r in srv.failed)
    assert len(fin) == len(arr) - n1
    s = summarize(fin, srv.failed, 0.05, 2)
    assert s["failed"] == n1 and s["completed"] == len(fin)


def test_oldest_request_first_across_rigs():
    be = FakeBackend(cost=[0.005, 0.005, 0.005], slot_bytes=[1, 1, 1])
    srv = Server(be, 3, hbm_budget=3, max_batch=1, n_streams=1)
    arr = [(0.0, 2, 0), (0.0001, 0, 0), (0.0002, 1, 0)]
    fin = srv.run(arr, realtime=True)
    order = [r.rig for r in sorted(fin, key=lambda r: r.start)]
    assert order == [2, 0, 1]


def test_poisson_arrivals_rates():
    arr = poisson_arrivals([50.0] * 6, 20.0, pool_size=16)
    assert 5600 < len(arr) < 6400
    assert all(arr[i][0] <= arr[i + 1][0] for i in range(len(arr) - 1))
