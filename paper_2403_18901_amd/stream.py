"""Streaming sliding-window decoding service.

Many logical blocks produce syndrome rounds over time; each block is decoded
window by window (Sec. III, Eq. 6-8): window k of an experiment becomes
decodable once its W rounds have arrived and window k - 1 has been committed.
The service batches every decodable window of every admitted experiment of
every block into one chained launch per code and tick: each experiment's
workgroup decodes all its windows whose rounds have arrived, strictly in
order, committing each into the experiment's device-resident detector record
and observable accumulator before the next reads its syndrome
(gdg_decode_chain; first, middle and last window shapes, a time-uniform DEM
giving all middle windows one graph). Finished experiments are evaluated
(Eq. 8-9). With chain=False a tick instead takes the next window of each
experiment only, in persistent multi-job launches followed by a commit.

Time is virtual: rounds arrive as a Poisson process per block in simulated
time, and each tick advances the clock by the measured device time of its
launches (HIP events), so latencies are queueing plus decode time on the GPU,
without the host's scheduling overhead (reported separately). Admission is by
device memory: a byte budget (by default a share of the free device memory
that hipMemGetInfo reports) is divided into experiment slots of each code --
its detector record and observable accumulator plus the per-window batch
buffers of one in-flight window -- and an experiment that starts while every
slot of its code is taken is rejected.

StreamScheduler is the host bookkeeping (numpy only); StreamingService drives
the library's kernels through the C ABI.
"""
import time

import numpy as np

from . import batched as B
from . import gdg as G


class StreamScheduler:
    """Arrivals, admission and window readiness for the blocks of one code.

    Block b's rounds arrive as a Poisson process of `rate` rounds per second;
    an experiment is n_rounds consecutive rounds; its window k (0 <= k < K,
    K = n_rounds - W + 1) needs rounds k .. k + W - 1 and the commit of window
    k - 1 of the same experiment (Sec. III). Experiments are independent
    decoding problems, so the admitted experiments of a block (and of all
    blocks) have their next windows decoded concurrently. An experiment is
    admitted at its first round if one of the n_slots device slots is free,
    else rejected.
    """

    def __init__(self, n_blocks, n_rounds, W, rate, n_slots, seed=0):
        self.nb, self.nR, self.W = n_blocks, n_rounds, W
        self.K = n_rounds - W + 1
        if self.K < 1:
            raise ValueError("fewer rounds than the window size")
        self.rate = float(rate)
        self.n_slots = n_slots
        self.rng = np.random.default_rng(seed)
        self.free = list(range(n_slots - 1, -1, -1))
        # arrival time of the first round of each block's next experiment
        self.t_first = self.rng.exponential(1.0 / self.rate, size=n_blocks)
        self.slot_block = np.full(n_slots, -1, np.int64)
        self.slot_k = np.zeros(n_slots, np.int64)
        self.slot_times = np.zeros((n_slots, n_rounds))
        self.slot_exp = np.full(n_slots, -1, np.int64)
        self.n_exp_started = 0
        self.n_admitted = 0
        self.n_rejected = 0
        self.next_exp_id = 0

    def _generate(self, now):
        """Every experiment whose first round arrives at or before `now`:
        (start times, blocks, round arrival times), in start order."""
        starts, blocks, times = [], [], []
        act = np.nonzero(self.t_first <= now)[0]
        while act.size:
            gaps = self.rng.exponential(1.0 / self.rate, size=(act.size, self.nR))
            t = self.t_first[act, None] + np.concatenate(
                [np.zeros((act.size, 1)), np.cumsum(gaps[:, 1:], axis=1)], axis=1)
            starts.append(t[:, 0])
            blocks.append(act)
            times.append(t)
            self.t_first[act] = t[:, -1] + gaps[:, 0]   # next experiment's first round
            act = act[self.t_first[act] <= now]
        if not starts:
            return np.zeros(0), np.zeros(0, np.int64), np.zeros((0, self.nR))
        s = np.concatenate(starts)
        order = np.argsort(s, kind="stable")
        return s[order], np.concatenate(blocks)[order], np.concatenate(times)[order]

    def advance_to(self, now):
        """Process arrivals up to `now`: experiments are admitted in start
        order while slots are free, the rest rejected. Returns (slots,
        experiment ids) newly admitted, ids consecutive."""
        s, b, t = self._generate(now)
        self.n_exp_started += s.size
        n = min(s.size, len(self.free))
        slots = np.array([self.free.pop() for _ in range(n)], np.int64)
        ids = np.arange(self.next_exp_id, self.next_exp_id + n, dtype=np.int64)
        self.slot_block[slots] = b[:n]
        self.slot_k[slots] = 0
        self.slot_times[slots] = t[:n]
        self.slot_exp[slots] = ids
        self.next_exp_id += n
        self.n_admitted += n
        self.n_rejected += s.size - n
        return slots, ids

    @property
    def pending(self):
        """Admitted, unfinished experiments of each block (slots, oldest first)."""
        out = [[] for _ in range(self.nb)]
        act = self.active()
        for slot in act[np.argsort(self.slot_exp[act], kind="stable")]:
            out[int(self.slot_block[slot])].append(int(slot))
        return out

    def active(self):
        """Slots of every admitted experiment not yet finished."""
        return np.nonzero(self.slot_block >= 0)[0].astype(np.int64)

    def avail_time(self, slots):
        k = self.slot_k[slots]
        return self.slot_times[slots, k + self.W - 1]

    def ready(self, now):
        """Slots whose next window is decodable at `now` (one window per
        experiment: its previous window is committed)."""
        h = self.active()
        if h.size == 0:
            return h
        return h[self.avail_time(h) <= now]

    def next_event(self):
        """Earliest time a next window becomes decodable (inf if none is waiting)."""
        h = self.active()
        if h.size == 0:
            return np.inf
        return float(self.avail_time(h).min())

    def next_start(self):
        """Arrival time of the next experiment start of any block."""
        return float(self.t_first.min())

    def chain_end(self, slots, now):
        """One past the last window of each slot whose rounds have all arrived
        at `now` (windows slot_k .. chain_end - 1 can be decoded in order)."""
        arrived = (self.slot_times[slots] <= now).sum(axis=1)
        return np.minimum(self.K, arrived - self.W + 1)

    def complete(self, slots, counts=1):
        """`counts` more windows of `slots` are committed; returns the slots
        whose experiment ended."""
        self.slot_k[slots] += counts
        done = slots[self.slot_k[slots] >= self.K]
        self.slot_block[done] = -1
        self.free.extend(int(x) for x in done)
        return done

    def backlog(self, now):
        """Windows whose rounds have arrived but that are not yet committed."""
        act = self.active()
        if act.size == 0:
            return 0
        arrived = (self.slot_times[act] <= now).sum(axis=1)
        ready = np.minimum(self.K, arrived - self.W + 1) - self.slot_k[act]
        return int(np.maximum(ready, 0).sum())


class _Code:
    """One code's windows (first, middle, last shapes), device sampler and,
    once sized, its experiment slots: the scheduler and the device-resident
    detector records and observable accumulators."""

    def __init__(self, dem, n_blocks, prm, W, rate, seed, stream_id, device):
        self.dem = dem
        self.n_blocks, self.W, self.rate = n_blocks, W, rate
        self.K = dem.n_rounds - W + 1
        self.w = dem.w
        self.n_rows, self.n_obs = dem.n_rows, max(dem.n_obs, 1)
        self.win = {0: G.Window(dem, 0, W, prm)}
        if self.K > 2:
            self.win[1] = G.Window(dem, 1, W, prm)
        if self.K > 1:
            self.win[self.K - 1] = G.Window(dem, self.K - 1, W, prm)
        self.m = self.win[0].m
        self.ddem = G.DeviceDem(dem)
        self.stream_id = stream_id
        self.seed = seed
        self.device = device
        self.fails = []     # (experiment id, failed)
        self.obs_out = {}   # experiment id -> observable accumulator after the last commit

    def slot_bytes(self, chain=True):
        """Device bytes of one experiment slot: its detector record and
        observable accumulator, plus its batch buffers in a tick (chained:
        correction scratch, every window's path metric and flags, two offsets
        and the window range; otherwise one window's syndrome, correction,
        path metric, flags and three offsets)."""
        n = max(w.n for w in self.win.values())
        if chain:
            return self.n_rows + self.n_obs + n + 12 * self.K + 2 * 8 + 2 * 4
        return self.n_rows + self.n_obs + self.m + n + 8 + 4 + 3 * 8

    def alloc(self, n_slots):
        import torch
        self.sched = StreamScheduler(self.n_blocks, self.dem.n_rounds, self.W, self.rate, n_slots,
                                     self.seed)
        self.det = torch.zeros((n_slots, self.n_rows), dtype=torch.uint8, device=self.device)
        self.obs = torch.zeros((n_slots, self.n_obs), dtype=torch.uint8, device=self.device)

    def shape_of(self, k):
        if k == 0:
            return 0
        if k == self.K - 1:
            return self.K - 1
        return 1


class StreamingService:
    """Continuous batching of the decodable windows of many blocks.

    codes: list of (dem, n_blocks). rate: rounds per second per block.
    mem_budget: device bytes for experiment slots (None: a quarter of the free
    device memory reported by hipMemGetInfo, at most 1 GiB), shared by the
    codes in proportion to n_blocks x slot_bytes. n_slots: a fixed slot count
    per code instead (tests).
    """

    def __init__(self, codes, prm, W=3, rate=1e6, n_slots=None, seed=0, plan=None,
                 device="cuda", mem_budget=None, chain=False, chain_max=0, decouple=False):
        """chain: decode through chained launches (gdg_decode_chain), at most
        chain_max windows of one experiment per tick (0: every decodable one);
        otherwise the next window of each experiment per tick. decouple: each
        code runs its own ticks on its own stream and clock, so one code's
        slow windows do not hold back the other's next tick."""
        import torch
        if chain and decouple:
            raise ValueError("decoupled ticks take the separate-launch policy")
        self.chain = chain
        self.chain_max = chain_max
        self.decouple = decouple
        self.codes = [_Code(dem, nb, prm, W, rate, seed + 7919 * i, i, device)
                      for i, (dem, nb) in enumerate(codes)]
        per = [c.slot_bytes(chain) for c in self.codes]
        if n_slots is None:
            if mem_budget is None:
                free, _ = torch.cuda.mem_get_info()   # hipMemGetInfo
                mem_budget = min(free // 4, 1 << 30)
            demand = sum(c.n_blocks * b for c, b in zip(self.codes, per))
        self.mem_budget = mem_budget
        self.slot_bytes = per
        for c, b in zip(self.codes, per):
            if n_slots is not None:
                c.alloc(n_slots)
            else:
                c.alloc(max(1, int(mem_budget * (c.n_blocks * b / demand) // b)))
        # one persistent launch per register tiling: windows of a small code do
        # not run in a larger code's tiling and LDS share; `plan` is one
        # LaunchPlan for every code or a list of them, one per code
        plan = plan or B.LaunchPlan(waves=4, wg_per_cu=0, split=True)
        self.plans = list(plan) if isinstance(plan, (list, tuple)) else [plan] * len(self.codes)
        if len(self.plans) != len(self.codes):
            raise ValueError("one launch plan per code")
        self.device = device
        self.streams = [torch.cuda.Stream(device=device) for _ in self.codes]
        self.now = 0.0
        self.latencies = []
        self.lat_code = []
        self.n_windows = 0
        self.n_ticks = 0
        self.device_s = 0.0
        self.host_s = 0.0
        self.batch_sizes = []

    def _admit(self, c, now):
        import torch
        slots, ids = c.sched.advance_to(now)
        if slots.size == 0:
            return
        # fresh syndromes of the admitted experiments (device sampler, experiment id
        # = shot index) written into their slots
        n = slots.size
        tmp_det = torch.empty((n, c.n_rows), dtype=torch.uint8, device=self.device)
        tmp_obs = torch.empty((n, c.n_obs), dtype=torch.uint8, device=self.device)
        assert ids[-1] - ids[0] == n - 1   # consecutive in admission order
        c.ddem.sample(n, seed=c.seed, stream=c.stream_id, shot0=int(ids[0]), device=self.device,
                      out=(tmp_det, tmp_obs))
        src = torch.arange(n, dtype=torch.int64, device=self.device)
        dst = torch.from_numpy(slots).to(self.device)
        G.copy_rows(tmp_det, src * c.n_rows, c.n_rows, c.det, dst * c.n_rows)
        G.copy_rows(tmp_obs, src * c.n_obs, c.n_obs, c.obs, dst * c.n_obs)

    def tick(self):
        """One batch: every decodable window of every admitted experiment
        (chained), or the next one of each (chain=False). Returns the number
        of windows decoded (0: nothing was ready at the current time)."""
        if self.chain:
            return self._tick_chain()
        import torch
        t_host = time.perf_counter()
        for c in self.codes:
            self._admit(c, self.now)
        groups = []   # (code, shape, slots)
        for c in self.codes:
            r = c.sched.ready(self.now)
            if r.size == 0:
                continue
            k = c.sched.slot_k[r]
            shapes = np.where(k == 0, 0, np.where(k == c.K - 1, c.K - 1, 1))
            for sh in np.unique(shapes):
                groups.append((c, int(sh), r[shapes == sh]))
        if not groups:
            self.host_s += time.perf_counter() - t_host
            return 0
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        main = torch.cuda.current_stream()
        e0.record(main)
        commits = []
        # each code's gathers, decode launches and commits on a stream of its
        # own: codes are independent, so their launches overlap (one code's
        # launch drains while the other's runs)
        for c in self.codes:
            mine = [(sh, slots) for cc, sh, slots in groups if cc is c]
            if not mine:
                continue
            st = self.streams[c.stream_id]
            st.wait_event(e0)
            with torch.cuda.stream(st):
                jobs, cm = [], []
                for sh, slots in mine:
                    win = c.win[sh]
                    k = c.sched.slot_k[slots]
                    off = torch.from_numpy(slots * c.n_rows + k * c.w).to(self.device)
                    n = slots.size
                    syn = torch.empty((n, win.m), dtype=torch.uint8, device=self.device)
                    G.copy_rows(c.det, off, win.m, syn)
                    outs = (torch.empty((n, win.n), dtype=torch.uint8, device=self.device),
                            torch.empty(n, dtype=torch.float64, device=self.device),
                            torch.empty(n, dtype=torch.int32, device=self.device))
                    jobs.append((win, syn, 0, outs))
                    obs_off = torch.from_numpy(slots * c.n_obs).to(self.device)
                    cm.append((c, win, outs[0], off, obs_off, slots))
                jobs.sort(key=lambda j: -(j[0].n_paths * j[0].n_act * j[1].shape[0]))
                for i in range(0, len(jobs), G.MAX_JOBS):
                    self.plans[c.stream_id].run(jobs[i:i + G.MAX_JOBS])
                for cc, win, ehat, off, obs_off, slots in cm:
                    win.commit_indexed(ehat, cc.det, off, cc.obs, obs_off)
                done = torch.cuda.Event()
                done.record(st)
            main.wait_event(done)
            commits.extend(cm)
        e1.record(main)
        e1.synchronize()
        dt = e0.elapsed_time(e1) * 1e-3
        self.device_s += dt
        done_t = self.now + dt
        nw = 0
        for c, win, ehat, off, obs_off, slots in commits:
            self.latencies.append(done_t - c.sched.avail_time(slots))
            self.lat_code.append(np.full(slots.size, c.stream_id))
            nw += slots.size
            done = c.sched.complete(slots)
            if done.size:
                self._evaluate(c, done)
        self.batch_sizes.append(nw)
        self.n_windows += nw
        self.n_ticks += 1
        self.now = done_t
        self.host_s += time.perf_counter() - t_host - dt
        return nw

    def _tick_chain(self):
        import torch
        t_host = time.perf_counter()
        for c in self.codes:
            self._admit(c, self.now)
        work = []   # (code, slots, first window, end)
        for c in self.codes:
            r = c.sched.ready(self.now)
            if r.size:
                kb = c.sched.slot_k[r].copy()
                ke = c.sched.chain_end(r, self.now)
                if self.chain_max > 0:
                    ke = np.minimum(ke, kb + self.chain_max)
                work.append((c, r, kb, ke))
        if not work:
            self.host_s += time.perf_counter() - t_host
            return 0
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        main = torch.cuda.current_stream()
        e0.record(main)
        # each code's chained launch on a stream of its own (codes are
        # independent: one code's launch drains while the other's runs)
        for c, slots, kb, ke in work:
            st = self.streams[c.stream_id]
            st.wait_event(e0)
            with torch.cuda.stream(st):
                dev = self.device
                n = slots.size
                nmax = max(w.n for w in c.win.values())
                G.decode_chain(c.win[0], c.win.get(1), c.win.get(c.K - 1), c.K,
                               torch.from_numpy(kb.astype(np.int32)).to(dev),
                               torch.from_numpy(ke.astype(np.int32)).to(dev), c.det,
                               torch.from_numpy(slots * c.n_rows).to(dev), c.obs,
                               torch.from_numpy(slots * c.n_obs).to(dev),
                               torch.empty((n, nmax), dtype=torch.uint8, device=dev),
                               torch.empty((n, c.K), dtype=torch.float64, device=dev),
                               torch.empty((n, c.K), dtype=torch.int32, device=dev))
                done = torch.cuda.Event()
                done.record(st)
            main.wait_event(done)
        e1.record(main)
        e1.synchronize()
        dt = e0.elapsed_time(e1) * 1e-3
        self.device_s += dt
        done_t = self.now + dt
        nw = 0
        for c, slots, kb, ke in work:
            cnt = ke - kb
            rows = np.repeat(np.arange(slots.size), cnt)
            ks = np.concatenate([np.arange(a, b) for a, b in zip(kb, ke)])
            self.latencies.append(done_t - c.sched.slot_times[slots[rows], ks + c.W - 1])
            self.lat_code.append(np.full(rows.size, c.stream_id))
            nw += int(cnt.sum())
            finished = c.sched.complete(slots, cnt)
            if finished.size:
                self._evaluate(c, finished)
        self.batch_sizes.append(nw)
        self.n_windows += nw
        self.n_ticks += 1
        self.now = done_t
        self.host_s += time.perf_counter() - t_host - dt
        return nw

    def _evaluate(self, c, slots):
        import torch
        n = slots.size
        sl = torch.from_numpy(slots).to(self.device)
        det = torch.empty((n, c.n_rows), dtype=torch.uint8, device=self.device)
        obs = torch.empty((n, c.n_obs), dtype=torch.uint8, device=self.device)
        G.copy_rows(c.det, sl * c.n_rows, c.n_rows, det)
        G.copy_rows(c.obs, sl * c.n_obs, c.n_obs, obs)
        f = G.evaluate(det, obs).cpu().numpy()
        o = obs.cpu().numpy()
        ids = c.sched.slot_exp[slots]
        c.fails.extend(zip(ids.tolist(), f.tolist()))
        for i, e in enumerate(ids.tolist()):
            c.obs_out[e] = o[i].copy()

    def _launch_code(self, c, now):
        """Decoupled ticks: admits and launches code c's decodable windows at
        its own clock `now`, everything on its stream. Returns the in-flight
        record, or None when nothing is ready."""
        import torch
        t_host = time.perf_counter()
        st = self.streams[c.stream_id]
        with torch.cuda.stream(st):
            self._admit(c, now)
            r = c.sched.ready(now)
            if r.size == 0:
                self.host_s += time.perf_counter() - t_host
                return None
            k_all = c.sched.slot_k[r]
            shapes = np.where(k_all == 0, 0, np.where(k_all == c.K - 1, c.K - 1, 1))
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            jobs, cm = [], []
            for sh in np.unique(shapes):
                slots = r[shapes == sh]
                win = c.win[int(sh)]
                k = c.sched.slot_k[slots]
                off = torch.from_numpy(slots * c.n_rows + k * c.w).to(self.device)
                n = slots.size
                syn = torch.empty((n, win.m), dtype=torch.uint8, device=self.device)
                G.copy_rows(c.det, off, win.m, syn)
                outs = (torch.empty((n, win.n), dtype=torch.uint8, device=self.device),
                        torch.empty(n, dtype=torch.float64, device=self.device),
                        torch.empty(n, dtype=torch.int32, device=self.device))
                jobs.append((win, syn, 0, outs))
                cm.append((win, outs[0], off, torch.from_numpy(slots * c.n_obs).to(self.device),
                           slots))
            jobs.sort(key=lambda j: -(j[0].n_paths * j[0].n_act * j[1].shape[0]))
            for i in range(0, len(jobs), G.MAX_JOBS):
                self.plans[c.stream_id].run(jobs[i:i + G.MAX_JOBS])
            for win, ehat, off, obs_off, slots in cm:
                win.commit_indexed(ehat, c.det, off, c.obs, obs_off)
            e1.record(st)
        self.host_s += time.perf_counter() - t_host
        return dict(c=c, e0=e0, e1=e1, start=now, cm=cm, keep=jobs)

    def _finish_code(self, rec, clocks, duration):
        """A decoupled tick completed: its code's clock advances by the tick's
        device time. Ticks started past `duration` only keep the device
        shared until every code has reached it; they are not counted."""
        c = rec["c"]
        dt = rec["e0"].elapsed_time(rec["e1"]) * 1e-3
        done_t = rec["start"] + dt
        count = rec["start"] < duration
        nw = 0
        for win, ehat, off, obs_off, slots in rec["cm"]:
            if count:
                self.latencies.append(done_t - c.sched.avail_time(slots))
                self.lat_code.append(np.full(slots.size, c.stream_id))
            nw += slots.size
            done = c.sched.complete(slots)
            if done.size:
                self._evaluate(c, done)
        if count:
            self.device_s += dt
            self.batch_sizes.append(nw)
            self.n_windows += nw
            self.n_ticks += 1
        clocks[c.stream_id] = done_t

    def _run_decoupled(self, duration, max_ticks=None):
        """Each code ticks on its own stream and clock (the launches of the
        codes overlap on the device, so each tick's measured time includes the
        sharing). Every code keeps the device busy until all clocks have
        passed `duration`; windows of ticks started before it are counted."""
        clocks = [self.now] * len(self.codes)
        inflight = {}
        while max_ticks is None or self.n_ticks < max_ticks:
            if all(t >= duration for t in clocks) and not inflight:
                break
            for c in self.codes:
                i = c.stream_id
                if i in inflight or all(t >= duration for t in clocks):
                    continue
                rec = self._launch_code(c, clocks[i])
                if rec is not None:
                    inflight[i] = rec
                    continue
                # idle: jump this code's clock to its next arrival
                nxt = min(c.sched.next_event(), c.sched.next_start())
                clocks[i] = max(clocks[i], min(nxt, duration) if clocks[i] < duration else nxt)
            if not inflight:
                continue
            done = None
            while done is None:   # the first launch in flight to complete
                for i, rec in inflight.items():
                    if rec["e1"].query():
                        done = i
                        break
            self._finish_code(inflight.pop(done), clocks, duration)
        for rec in inflight.values():
            rec["e1"].synchronize()
            self._finish_code(rec, clocks, duration)
        self.now = duration
        return self.report(duration)

    def run(self, duration, max_ticks=None):
        """Runs until the virtual clock passes `duration` seconds."""
        if self.decouple:
            return self._run_decoupled(duration, max_ticks)
        while self.now < duration and (max_ticks is None or self.n_ticks < max_ticks):
            if self.tick() == 0:
                # idle: jump to the next arrival that can make a window ready
                nxt = min(min(c.sched.next_event() for c in self.codes),
                          min(c.sched.next_start() for c in self.codes))
                self.now = max(self.now, min(nxt, duration))
                if nxt >= duration:
                    break
        return self.report(duration)

    def report(self, duration):
        lat = np.concatenate(self.latencies) if self.latencies else np.zeros(0)
        code = np.concatenate(self.lat_code) if self.lat_code else np.zeros(0, np.int64)
        by_code = {}
        for c in self.codes:
            x = lat[code == c.stream_id]
            by_code[c.dem.name.split()[0]] = {
                "windows": int(x.size),
                "p50": float(np.percentile(x, 50) * 1e3) if x.size else None,
                "p99": float(np.percentile(x, 99) * 1e3) if x.size else None}
        span = max(self.now, 1e-12)
        offered = sum(c.sched.nb * c.sched.rate * c.K / c.sched.nR for c in self.codes)
        backlog = sum(c.sched.backlog(self.now) for c in self.codes)
        return {
            "virtual_s": self.now,
            "windows": int(self.n_windows),
            "windows_per_s": self.n_windows / span,
            "offered_windows_per_s": offered,
            "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
                           "p99": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
                           "max": float(lat.max() * 1e3) if lat.size else None},
            "latency_ms_by_code": by_code,
            "backlog_windows": int(backlog),
            "backlog_growth_per_s": backlog / span,
            "mem_budget_bytes": int(self.mem_budget) if self.mem_budget is not None else None,
            "slots": [int(c.sched.n_slots) for c in self.codes],
            "slot_bytes": [int(b) for b in self.slot_bytes],
            "experiments_started": int(sum(c.sched.n_exp_started for c in self.codes)),
            "admitted": int(sum(c.sched.n_admitted for c in self.codes)),
            "rejected": int(sum(c.sched.n_rejected for c in self.codes)),
            "ticks": int(self.n_ticks),
            "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
            "device_busy_frac": self.device_s / span,
            "host_ms_per_tick": self.host_s * 1e3 / max(self.n_ticks, 1),
            "failures": int(sum(f for c in self.codes for _, f in c.fails)),
            "experiments_done": int(sum(len(c.fails) for c in self.codes)),
        }
