"""Host bookkeeping of the streaming service (arrivals, admission, readiness)."""
import numpy as np

from paper_2403_18901_amd.stream import StreamScheduler


def test_poisson_experiment_starts():
    """Experiments are n_rounds consecutive rounds of a Poisson round stream:
    starts by time T are about rate * T / n_rounds per block."""
    s = StreamScheduler(50, 13, 3, rate=1e4, n_slots=10**6, seed=3)
    T = 0.5
    s.advance_to(T)
    expect = 50 * 1e4 * T / 13
    assert abs(s.n_exp_started - expect) < 5 * np.sqrt(expect)
    assert s.n_rejected == 0 and s.n_admitted == s.n_exp_started
    # round times of every admitted experiment are increasing and start <= T
    used = s.slot_block >= 0
    t = s.slot_times[used]
    assert (np.diff(t, axis=1) > 0).all() and (t[:, 0] <= T).all()


def test_admission_cap_and_rejections():
    s = StreamScheduler(8, 7, 3, rate=1e3, n_slots=3, seed=1)
    slots, ids = s.advance_to(0.2)
    assert slots.size == 3 and list(ids) == [0, 1, 2]
    assert s.n_admitted == 3 and s.n_rejected == s.n_exp_started - 3
    assert sum(len(p) for p in s.pending) == 3


def test_windows_in_order_per_experiment():
    """An experiment's window k is ready only when its round k+W-1 has arrived
    and window k-1 is committed, one window per experiment at a time, and the
    slot frees after K windows."""
    s = StreamScheduler(1, 6, 3, rate=100.0, n_slots=2, seed=0)
    now = 0.0
    s.advance_to(now)
    while not any(s.pending):
        now = s.next_start()
        s.advance_to(now)
    slot = s.pending[0][0]
    times = s.slot_times[slot].copy()
    K = s.K
    for k in range(K):
        avail = times[k + 2]
        assert s.ready(avail - 1e-12).size == 0 or s.slot_k[slot] != k
        r = s.ready(avail)
        assert list(r) == [slot] and s.slot_k[slot] == k
        assert abs(s.next_event() - avail) < 1e-15
        done = s.complete(r)
        assert (done.size == 1) == (k == K - 1)
    assert s.slot_block[slot] == -1 and slot in s.free


def test_fake_service_drains_every_admitted_experiment():
    """Constant-time fake decode ticks: every admitted experiment completes,
    latencies are non-negative, and the backlog is empty at the end."""
    s = StreamScheduler(5, 8, 3, rate=2e3, n_slots=7, seed=4)
    now, lat, done = 0.0, [], 0
    while now < 0.3 or any(s.pending):
        if now < 0.3:
            s.advance_to(now)
        r = s.ready(now)
        if r.size == 0:
            nxt = s.next_event()
            if now < 0.3:
                nxt = min(nxt, s.next_start())
            now = max(now, nxt)
            continue
        now += 1e-4
        lat.extend((now - s.avail_time(r)).tolist())
        done += s.complete(r).size
    assert done == s.n_admitted and min(lat) >= 0.0
    assert s.backlog(now) == 0


def test_experiments_of_a_block_decode_concurrently():
    """A block's later experiments do not wait for its earlier ones: once
    their rounds have arrived, the next windows of all of them are ready in the
    same tick (each experiment still one window at a time, in order)."""
    s = StreamScheduler(1, 6, 3, rate=1e5, n_slots=8, seed=2)
    s.advance_to(1e-3)                        # about 16 experiments started, 8 admitted
    assert s.n_admitted == 8 and s.n_rejected > 0
    r = s.ready(1.0)
    assert r.size == 8                        # every admitted experiment has window 0 ready
    s.complete(r)
    assert (s.slot_k[r] == 1).all()
    r2 = s.ready(1.0)
    assert sorted(r2.tolist()) == sorted(r.tolist())
    for _ in range(s.K - 1):
        s.complete(s.ready(1.0))
    assert s.active().size == 0 and len(s.free) == 8 and not any(s.pending)


def test_chain_end_counts_the_windows_whose_rounds_arrived():
    """Window k of an experiment needs rounds k .. k + W - 1: at a time when
    r rounds have arrived, windows slot_k .. r - W are decodable in order
    (capped at K), and completing several at once advances the slot by that
    many and frees it at the end."""
    s = StreamScheduler(n_blocks=1, n_rounds=7, W=3, rate=1e3, n_slots=2, seed=3)
    slots, _ = s.advance_to(s.t_first[0])
    t = s.slot_times[slots[0]]
    assert s.chain_end(slots, t[1]).tolist() == [0]     # two rounds: nothing yet
    assert s.chain_end(slots, t[2]).tolist() == [1]
    assert s.chain_end(slots, t[5]).tolist() == [4]
    assert s.chain_end(slots, t[6] + 1.0).tolist() == [5]   # K = 5
    done = s.complete(slots, np.array([3]))
    assert done.size == 0 and s.slot_k[slots[0]] == 3
    done = s.complete(slots, np.array([2]))
    assert done.tolist() == slots.tolist() and slots[0] in s.free
