"""Streaming sliding-window decoding service.

Many logical blocks produce syndrome rounds over time; each block is decoded
window by window (Sec. III, Eq. 6-8): window k of an experiment becomes
decodable once its W rounds have arrived and window k - 1 has been committed.
The service batches every decodable window of every block into one persistent
multi-job launch per tick (one job per code and window shape: first, middle,
last window of an experiment; a time-uniform DEM gives all middle windows one
graph), commits each window into its block's device-resident detector record
and observable accumulator, and evaluates experiments that finished (Eq. 8-9).

Time is virtual: rounds arrive as a Poisson process per block in simulated
time, and each tick advances the clock by the measured device time of its
launches (HIP events), so latencies are queueing plus decode time on the GPU,
without the host's scheduling overhead (reported separately). Admission: an
experiment that starts while every device slot of its code is taken (the
memory budget) is rejected.

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
    K = n_rounds - W + 1) needs rounds k .. k + W - 1. A block decodes its
    experiments in order, one window at a time. An experiment is admitted at
    its first round if one of the n_slots device slots is free, else rejected.
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
        self.pending = [[] for _ in range(n_blocks)]   # admitted experiments, oldest first
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
        """Process arrivals up to `now`; returns (slots, experiment ids) newly
        admitted, ids consecutive."""
        s, b, t = self._generate(now)
        self.n_exp_started += s.size
        new_slots, new_ids = [], []
        for i in range(s.size):
            if not self.free:
                self.n_rejected += 1
                continue
            slot = self.free.pop()
            blk = int(b[i])
            self.slot_block[slot] = blk
            self.slot_k[slot] = 0
            self.slot_times[slot] = t[i]
            self.slot_exp[slot] = self.next_exp_id
            new_ids.append(self.next_exp_id)
            self.next_exp_id += 1
            self.pending[blk].append(slot)
            new_slots.append(slot)
            self.n_admitted += 1
        return np.array(new_slots, np.int64), np.array(new_ids, np.int64)

    def heads(self):
        """Slot of each block's oldest admitted experiment (or none)."""
        return np.array([p[0] for p in self.pending if p], np.int64)

    def avail_time(self, slots):
        k = self.slot_k[slots]
        return self.slot_times[slots, k + self.W - 1]

    def ready(self, now):
        """Slots whose next window is decodable at `now` (one per block at most)."""
        h = self.heads()
        if h.size == 0:
            return h
        return h[self.avail_time(h) <= now]

    def next_event(self):
        """Earliest time a head window becomes decodable (inf if none is waiting)."""
        h = self.heads()
        if h.size == 0:
            return np.inf
        return float(self.avail_time(h).min())

    def next_start(self):
        """Arrival time of the next experiment start of any block."""
        return float(self.t_first.min())

    def complete(self, slots):
        """Windows of `slots` are committed; returns the slots whose experiment ended."""
        self.slot_k[slots] += 1
        done = slots[self.slot_k[slots] >= self.K]
        for slot in done:
            blk = int(self.slot_block[slot])
            assert self.pending[blk] and self.pending[blk][0] == slot
            self.pending[blk].pop(0)
            self.slot_block[slot] = -1
            self.free.append(int(slot))
        return done

    def backlog(self, now):
        """Windows whose rounds have arrived but that are not yet committed."""
        n = 0
        for slot in range(self.n_slots):
            if self.slot_block[slot] < 0:
                continue
            arrived = int(np.searchsorted(self.slot_times[slot], now, side="right"))
            n += max(0, min(self.K, arrived - self.W + 1) - int(self.slot_k[slot]))
        return n


class _Code:
    def __init__(self, dem, n_blocks, prm, W, rate, n_slots, seed, stream_id, device):
        import torch
        self.dem = dem
        self.sched = StreamScheduler(n_blocks, dem.n_rounds, W, rate, n_slots, seed)
        self.K = self.sched.K
        self.w = dem.w
        self.n_rows, self.n_obs = dem.n_rows, max(dem.n_obs, 1)
        self.win = {0: G.Window(dem, 0, W, prm)}
        if self.K > 2:
            self.win[1] = G.Window(dem, 1, W, prm)
        if self.K > 1:
            self.win[self.K - 1] = G.Window(dem, self.K - 1, W, prm)
        self.m = self.win[0].m
        self.ddem = G.DeviceDem(dem)
        self.det = torch.zeros((n_slots, self.n_rows), dtype=torch.uint8, device=device)
        self.obs = torch.zeros((n_slots, self.n_obs), dtype=torch.uint8, device=device)
        self.stream_id = stream_id
        self.seed = seed
        self.device = device
        self.fails = []     # (experiment id, failed)
        self.obs_out = {}   # experiment id -> observable accumulator after the last commit

    def shape_of(self, k):
        if k == 0:
            return 0
        if k == self.K - 1:
            return self.K - 1
        return 1


class StreamingService:
    """Continuous batching of the decodable windows of many blocks.

    codes: list of (dem, n_blocks). rate: rounds per second per block.
    n_slots: device slots (concurrent experiments) per code, the memory budget.
    """

    def __init__(self, codes, prm, W=3, rate=1e6, n_slots=None, seed=0, plan=None,
                 device="cuda"):
        self.codes = []
        for i, (dem, nb) in enumerate(codes):
            ns = n_slots if n_slots is not None else 2 * nb
            self.codes.append(_Code(dem, nb, prm, W, rate, ns, seed + 7919 * i, i, device))
        self.plan = plan or B.LaunchPlan(waves=4, wg_per_cu=0, split=False)
        self.device = device
        self.now = 0.0
        self.latencies = []
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
        """One batch: every decodable head window of every block. Returns the
        number of windows decoded (0: nothing was ready at the current time)."""
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
            shapes = np.array([c.shape_of(int(x)) for x in k])
            for sh in np.unique(shapes):
                groups.append((c, int(sh), r[shapes == sh]))
        if not groups:
            self.host_s += time.perf_counter() - t_host
            return 0
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        jobs, commits = [], []
        e0.record()
        for c, sh, slots in groups:
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
            commits.append((c, win, outs[0], off, obs_off, slots))
        jobs.sort(key=lambda j: -(j[0].n_paths * j[0].n_act * j[1].shape[0]))
        for i in range(0, len(jobs), G.MAX_JOBS):
            self.plan.run(jobs[i:i + G.MAX_JOBS])
        for c, win, ehat, off, obs_off, slots in commits:
            win.commit_indexed(ehat, c.det, off, c.obs, obs_off)
        e1.record()
        e1.synchronize()
        dt = e0.elapsed_time(e1) * 1e-3
        self.device_s += dt
        done_t = self.now + dt
        nw = 0
        for c, win, ehat, off, obs_off, slots in commits:
            self.latencies.append(done_t - c.sched.avail_time(slots))
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

    def run(self, duration, max_ticks=None):
        """Runs until the virtual clock passes `duration` seconds."""
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
            "backlog_windows": int(backlog),
            "backlog_growth_per_s": backlog / span,
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
