"""Mixed-size batched decoding and the launch autotuner.

Several BB codes (windows of uneven size) are decoded together: at window step
k every code still in its window range contributes one job, and the jobs share
one persistent launch (`gdg_decode_jobs`). The autotuner times candidate launch
shapes on a sample of the real jobs and keeps the fastest:

* wavefronts per workgroup (each wavefront runs whole decision paths),
* persistent grid size (workgroups per CU x CU count, or one per shot),
* schedule: all jobs in one launch, or one launch per kernel register tiling
  (so small codes do not run in the largest code's tiling), each tiling's
  launch then with a shape of its own: the tilings' launches run one after
  another, so the tuner times each tiling's jobs alone, composes the fastest
  shape per tiling and times the composed plan as well.
"""
from __future__ import annotations

import itertools
import time

import torch

from . import gdg as G

N_CU = 256


def _bucket(w) -> int:
    """The kernel's register tiling for a window (VNs per lane)."""
    na = w.n_act
    for b, cap in enumerate((384, 448, 512, 896)):
        if na <= cap:
            return b
    return 4


class LaunchPlan:
    """How a set of jobs is launched: waves, grid, and grouping into launches.
    per_bucket ({tiling: (waves, wg_per_cu)}, split plans only) overrides the
    shape of that tiling's launch."""

    def __init__(self, waves=4, wg_per_cu=0, split=False, per_bucket=None):
        self.waves = waves
        self.wg_per_cu = wg_per_cu      # 0: one workgroup per shot
        self.split = split              # one launch per register tiling
        self.per_bucket = dict(per_bucket or {}) if split else {}

    def __repr__(self):
        extra = f", per_bucket={self.per_bucket}" if self.per_bucket else ""
        return (f"LaunchPlan(waves={self.waves}, wg_per_cu={self.wg_per_cu}, "
                f"split={self.split}{extra})")

    def key(self):
        return (self.waves, self.wg_per_cu, self.split, tuple(sorted(self.per_bucket.items())))

    def run(self, jobs):
        """jobs: list of (Window, syn, offset, outs), costliest first."""
        groups = [(None, jobs)]
        if self.split:
            by = {}
            for j in jobs:
                by.setdefault(_bucket(j[0]), []).append(j)
            groups = [(b, by[b]) for b in sorted(by, reverse=True)]
        for b, grp in groups:
            waves, wpc = self.per_bucket.get(b, (self.waves, self.wg_per_cu))
            G.decode_jobs(grp, waves=waves, workgroups=wpc * N_CU if wpc else 0)


def candidate_plans(windows):
    limit = 160 * 1024
    plans = []
    for waves, wpc, split in itertools.product((2, 4, 8), (0, 1, 2, 3, 4), (False, True)):
        if G.jobs_lds_bytes(windows, waves) > limit:
            continue
        if wpc and G.jobs_lds_bytes(windows, waves) * wpc > limit:
            continue   # that many workgroups cannot be resident per CU
        if split and len({_bucket(w) for w in windows}) == 1:
            continue
        plans.append(LaunchPlan(waves, wpc, split))
    return plans


_cache = {}


def autotune(jobs, reps: int = 2, plans=None, verbose: bool = False):
    """Times every candidate plan on `jobs` (decoded in place into their output
    buffers; inputs are not modified) and returns (best plan, timings)."""
    windows = [j[0] for j in jobs]
    key = tuple((w.m, w.n, w.n_act, w.n_paths, j[1].shape[0]) for w, j in zip(windows, jobs))
    if key in _cache and plans is None:
        return _cache[key]
    composed = plans is None
    plans = plans or candidate_plans(windows)
    timings = {}

    def time_plan(p, js):
        p.run(js)                         # warm-up (LDS attribute, code load)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            p.run(js)
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    for p in plans:
        timings[p.key()] = time_plan(p, jobs)
        if verbose:
            print(f"  {p}: {timings[p.key()]:.2f} ms", flush=True)
    by = {}
    for j in jobs:
        by.setdefault(_bucket(j[0]), []).append(j)
    if composed and len(by) > 1:
        # each tiling's launch on its own, then the composition of the fastest
        per = {}
        for b, grp in by.items():
            sub = {}
            for p in candidate_plans([j[0] for j in grp]):
                if not p.split:
                    sub[(p.waves, p.wg_per_cu)] = time_plan(p, grp)
            per[b] = min(sub, key=sub.get)
        comp = LaunchPlan(split=True, per_bucket=per)
        plans = list(plans) + [comp]
        timings[comp.key()] = time_plan(comp, jobs)
        if verbose:
            print(f"  {comp}: {timings[comp.key()]:.2f} ms", flush=True)
    best_key = min(timings, key=timings.get)
    best = next(p for p in plans if p.key() == best_key)
    _cache[key] = (best, timings)
    return best, timings


class MixedDecoder:
    """(W,1) sliding-window GDG over several DEMs (codes) at once: window step k
    decodes every code's window k in one persistent launch, then commits each."""

    def __init__(self, dems, prms, W: int = 3):
        self.dems = list(dems)
        self.decoders = [G.SlidingWindowDecoder(d, p, W=W) for d, p in zip(self.dems, prms)]
        self.steps = max(d.n_windows for d in self.decoders)
        self.plan = LaunchPlan()

    def _jobs(self, k, dets, outs):
        jobs = []
        for c, (dec, det) in enumerate(zip(self.decoders, dets)):
            if k < dec.n_windows:
                w = dec.windows[k]
                jobs.append((w, det, w.row0, outs[c][k]))
        # costliest first: paths x truncated columns per shot
        jobs.sort(key=lambda j: -(j[0].n_paths * j[0].n_act))
        return jobs

    def alloc(self, dets):
        outs = []
        for dec, det in zip(self.decoders, dets):
            ns = det.shape[0]
            outs.append([(torch.empty((ns, w.n), dtype=torch.uint8, device=det.device),
                          torch.empty(ns, dtype=torch.float64, device=det.device),
                          torch.empty(ns, dtype=torch.int32, device=det.device))
                         for w in dec.windows])
        return outs

    def tune(self, dets, reps: int = 2, verbose: bool = False):
        """Autotunes on a copy of the first window step's jobs."""
        scratch = [d.clone() for d in dets]
        outs = self.alloc(scratch)
        self.plan, timings = autotune(self._jobs(0, scratch, outs), reps=reps, verbose=verbose)
        return self.plan, timings

    def decode(self, dets, obss, outs=None):
        """Decodes in place (detectors become residuals, observables accumulate
        L e); returns per-code failure flags."""
        outs = outs or self.alloc(dets)
        for k in range(self.steps):
            jobs = self._jobs(k, dets, outs)
            self.plan.run(jobs)
            for c, (dec, det, obs) in enumerate(zip(self.decoders, dets, obss)):
                if k < dec.n_windows:
                    ehat = outs[c][k][0]
                    dec.windows[k].commit(ehat, det, obs)
        return [G.evaluate(d, o) for d, o in zip(dets, obss)]
