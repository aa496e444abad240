"""ctypes binding of the FP64 CPU oracle (gdg_oracle.cpp).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU
baseline use this module. It does not import the GPU package, and the GPU
package never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gdg_oracle.cpp")
LIB = os.path.join(HERE, "libgdg_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (plain C++17, -O2)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread",
                               SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


class Params(C.Structure):
    _fields_ = [("alpha", C.c_double), ("clip", C.c_double), ("iters_per_step", C.c_int),
                ("pre_iters", C.c_int), ("trunc_factor", C.c_int), ("g", C.c_int),
                ("dmax_main", C.c_int), ("extra_steps", C.c_int),
                ("side_max_depth", C.c_int), ("low_error", C.c_int),
                ("sum_product", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("n_paths", C.c_int), ("converged_path", C.c_int),
                ("pre_converged", C.c_int), ("bp_iters", C.c_longlong),
                ("edge_iters", C.c_longlong), ("steps_main", C.c_int)]


def params(alpha=1.0, clip=50.0, iters_per_step=6, pre_iters=0, trunc_factor=2, g=0,
           dmax_main=25, extra_steps=10, side_max_depth=0, low_error=1, sum_product=0):
    return Params(alpha, clip, iters_per_step, pre_iters, trunc_factor, g, dmax_main,
                  extra_steps, side_max_depth, low_error, sum_product)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        i32 = C.c_int
        L.orc_window_new.restype = P
        L.orc_window_new.argtypes = [i32] * 5 + [P] * 5 + [i32, i32, i32]
        L.orc_window_free.argtypes = [P]
        L.orc_window_dims.argtypes = [P, P]
        L.orc_window_export.argtypes = [P] * 6
        L.orc_window_bp.argtypes = [P, P, P, i32, P, P, P]
        L.orc_window_bp.restype = i32
        L.orc_window_decode.argtypes = [P, P, i32, P, P, P, P, P, P, i32, P, i32, i32, P, P,
                                        i32, i32, P, P, P]
        L.orc_warm_map.argtypes = [P, P, P]
        L.orc_warm_map.restype = i32
        L.orc_window_replay.argtypes = [P, P, P, P, i32, P, P, i32] + [P] * 11 + [i32, P, P, P, P, P, P]
        L.orc_window_replay.restype = i32
        L.orc_decode_shots.argtypes = [i32] * 5 + [P] * 5 + [i32, P, i32] + [P] * 8 + [i32] * 8
        L.orc_decode_shots.restype = i32
        L.orc_select_vn.argtypes = [i32, P, P, P, P, i32, i32, i32, P, P]
        L.orc_select_vn.restype = i32
        L.orc_agg_dec.argtypes = [P, i32, i32, i32]
        L.orc_agg_dec.restype = i32
        L.orc_path_value.argtypes = [P, i32, i32, i32, P, P]
        L.orc_path_value.restype = i32
        L.orc_n_paths.argtypes = [P]
        L.orc_n_paths.restype = i32
        L.orc_peel.argtypes = [i32, i32, P, P, P]
        L.orc_peel.restype = i32
        L.orc_dense_bp.argtypes = [i32, i32, P, P, P, P, i32, P]
        L.orc_dense_gdg.argtypes = [i32, i32, P, P, P, P, P, P]
        L.orc_dense_gdg.restype = C.c_double
        L.orc_window_osd.argtypes = [P, P, i32, P, i32, i32, i32, i32, P, P, P, P, P, P, i32]
        L.orc_dense_osd.argtypes = [i32, i32, P, P, P, P, i32, i32, i32, i32, P, P]
        L.orc_dense_osd.restype = C.c_double
        L.orc_dense_window.argtypes = [i32, i32, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_dense_window.restype = C.c_double
        L.orc_dense_path_probe.argtypes = [i32, i32, P, P, P, P, i32, i32] + [P] * 7
        L.orc_dense_path_probe.restype = i32
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _dem_args(dem):
    arrs = [np.ascontiguousarray(dem.h_ptr, np.int32), np.ascontiguousarray(dem.h_idx, np.int32),
            np.ascontiguousarray(dem.l_ptr, np.int32), np.ascontiguousarray(dem.l_idx, np.int32),
            np.ascontiguousarray(dem.priors, np.float64)]
    return arrs


def default_threads():
    return max(1, len(os.sched_getaffinity(0)))


def n_windows(n_rounds, W, F=1):
    """Windows of a (W,F) sliding window over n_rounds detector rounds."""
    return 1 if n_rounds <= W else 1 + (n_rounds - W + F - 1) // F


class OracleWindow:
    """Window k of a (W,F) sliding window, built by the oracle."""

    def __init__(self, dem, k, W=3, F=1):
        self._keep = _dem_args(dem)
        self.h = lib().orc_window_new(dem.n_rows, dem.n_cols, dem.n_obs, dem.w, dem.n_rounds,
                                      *[_p(a) for a in self._keep], k, W, F)
        if not self.h:
            raise ValueError("window build failed")
        dims = np.zeros(4, np.int32)
        lib().orc_window_dims(self.h, _p(dims))
        self.m, self.n, self.n_edges, self.row0 = [int(x) for x in dims]
        self.k = k
        self.W = W

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_window_free(self.h)
            self.h = None

    def export(self):
        dense = np.zeros((self.m, self.n), np.uint8)
        src = np.zeros(self.n, np.int32)
        prior = np.zeros(self.n, np.float64)
        llr = np.zeros(self.n, np.float64)
        commit = np.zeros(self.n, np.uint8)
        lib().orc_window_export(self.h, _p(dense), _p(src), _p(prior), _p(llr), _p(commit))
        return dict(H=dense, src=src, prior=prior, llr=llr, commit=commit)

    def bp(self, prm, syn, n_iters, with_cn_min=False, warm_in=None):
        """Flooding BP on the whole window, every iteration's posteriors; warm_in
        (per edge, NaN: none) starts it as the warm-started preprocessing."""
        syn = np.ascontiguousarray(syn, np.uint8)
        post = np.zeros((n_iters, self.n), np.float64)
        cmin = np.zeros((n_iters, self.m), np.float64) if with_cn_min else None
        wi = None if warm_in is None else np.ascontiguousarray(warm_in, np.float64)
        first = lib().orc_window_bp(self.h, C.byref(prm), _p(syn), n_iters, _p(post), _p(cmin),
                                    _p(wi))
        if with_cn_min:
            return post, first, cmin
        return post, first

    def decode(self, prm, syn, n_threads=None, logs=False, log_cap=32, warm_in=None,
               warm_out=False):
        """Window decode; warm_in [n_shots][edges] (row-major window edges, NaN
        for edges the previous window lacks) starts the preprocessing BP from
        those CN-to-VN messages, warm_out=True returns the messages this window
        hands over (key "warm_out")."""
        syn = np.ascontiguousarray(syn, np.uint8).reshape(-1, self.m)
        ns = syn.shape[0]
        ne = self.n_edges if (warm_in is not None or warm_out) else 0
        wi = None if warm_in is None else np.ascontiguousarray(warm_in, np.float64).reshape(ns, ne)
        wo = np.zeros((ns, ne), np.float64) if warm_out else None
        e = np.zeros((ns, self.n), np.uint8)
        pm = np.zeros(ns, np.float64)
        flags = np.zeros(ns, np.int32)
        stats = (Stats * ns)()
        npaths = lib().orc_n_paths(C.byref(prm))
        sel = dec = ends = post = None
        sel_cap = self.n
        if logs:
            sel = np.zeros((ns, sel_cap), np.int32)
            dec = np.zeros((ns, npaths, log_cap, 3), np.int32)
            ends = np.zeros((ns, npaths, 2), np.int32)
            post = np.zeros((ns, self.n), np.float64)
        lsum = np.zeros((ns, self.n), np.float64) if logs else None
        lib().orc_window_decode(self.h, C.byref(prm), ns, _p(syn), _p(e), _p(pm), _p(flags),
                                C.cast(stats, C.c_void_p), _p(sel), sel_cap if logs else 0,
                                _p(dec), npaths if logs else 0, log_cap, _p(ends), _p(post),
                                self.n if logs else 0, n_threads or default_threads(), _p(wi),
                                _p(wo), _p(lsum))
        out = dict(e=e, pm=pm, flags=flags,
                   edge_iters=np.array([s.edge_iters for s in stats], np.int64),
                   bp_iters=np.array([s.bp_iters for s in stats], np.int64),
                   converged_path=np.array([s.converged_path for s in stats], np.int32),
                   steps_main=np.array([s.steps_main for s in stats], np.int32),
                   pre_converged=np.array([s.pre_converged for s in stats], np.int32))
        if logs:
            out.update(sel=sel, dec=dec, ends=ends, first_post=post, lsum=lsum)
        if warm_out:
            out["warm_out"] = wo
        return out

    def warm_map(self, prev):
        """For each edge of this window, the edge of window `prev` it continues
        (same detector row and DEM column) or -1."""
        mp = np.zeros(self.n_edges, np.int32)
        lib().orc_warm_map(prev.h, self.h, _p(mp))
        return mp

    def osd(self, prm, syn, n_iters=200, cs=True, lam=10, n_keep=0, forced_order=None,
            n_threads=None):
        """BP + OSD-CS(lam) (or OSD-0 with cs=False) on window syndromes; n_keep
        > 0 keeps only the first n_keep ranked columns. Returns dict(e, pm,
        flags, order (-1 rows where BP met the syndrome), bp_iters)."""
        syn = np.ascontiguousarray(syn, np.uint8).reshape(-1, self.m)
        ns = syn.shape[0]
        e = np.zeros((ns, self.n), np.uint8)
        pm = np.zeros(ns, np.float64)
        fl = np.zeros(ns, np.int32)
        order = np.zeros((ns, self.n), np.int32)
        it = np.zeros(ns, np.int32)
        fo = None if forced_order is None else np.ascontiguousarray(forced_order, np.int32)
        lib().orc_window_osd(self.h, C.byref(prm), ns, _p(syn), n_iters, int(cs), lam, n_keep,
                             _p(fo), _p(e), _p(pm), _p(fl), _p(order), _p(it),
                             n_threads or default_threads())
        return dict(e=e, pm=pm, flags=fl, order=order, bp_iters=it)

    def replay(self, prm, syn, forced_sel, path_id, forced_g, forced_v, max_steps=64):
        syn = np.ascontiguousarray(syn, np.uint8)
        fs = None if forced_sel is None else np.ascontiguousarray(forced_sel, np.int32)
        fg = np.ascontiguousarray(forced_g, np.int32)
        fv = np.ascontiguousarray(forced_v, np.int32)
        own_g = np.full(max_steps, -1, np.int32)
        own_v = np.full(max_steps, -1, np.int32)
        own_key = np.full(max_steps, np.nan)
        forced_key = np.full(max_steps, np.nan)
        own_class = np.full(max_steps, -1, np.int32)
        forced_class = np.full(max_steps, -1, np.int32)
        lsum = np.zeros(self.n, np.float64)
        e = np.zeros(self.n, np.uint8)
        pm = np.zeros(1, np.float64)
        n_sub = self.n if prm.pre_iters == 0 else min(self.n, prm.trunc_factor * self.m)
        step_lsum = np.full((max_steps, n_sub), np.nan)
        step_min = np.full(max_steps, np.nan)
        own_hmax = np.full(max_steps, np.nan)
        forced_hmax = np.full(max_steps, np.nan)
        step_min_post = np.full(max_steps, np.nan)
        step_nagg = np.full(max_steps, -1, np.int32)
        step_agg_margin = np.full(max_steps, np.nan)
        first_post = np.full(n_sub, np.nan)
        r = lib().orc_window_replay(self.h, C.byref(prm), _p(syn), _p(fs), path_id, _p(fg),
                                    _p(fv), len(fg), _p(own_g), _p(own_v), _p(own_key),
                                    _p(forced_key), _p(own_class), _p(forced_class), _p(lsum),
                                    _p(e), _p(pm), _p(step_lsum), _p(step_min), max_steps,
                                    _p(own_hmax), _p(forced_hmax), _p(step_min_post),
                                    _p(step_nagg), _p(step_agg_margin), _p(first_post))
        return dict(code=r, steps=r // 8, end=r % 8, own_g=own_g, own_v=own_v,
                    own_key=own_key, forced_key=forced_key, own_class=own_class,
                    forced_class=forced_class, lsum=lsum, e=e, pm=float(pm[0]),
                    step_lsum=step_lsum, step_min_msg=step_min, own_hmax=own_hmax,
                    forced_hmax=forced_hmax, step_min_post=step_min_post,
                    step_nagg=step_nagg, step_agg_margin=step_agg_margin,
                    first_post=first_post)


def decode_shots(dem, W, prm, det, obs, n_threads=None, max_windows=-1, F=1, osd=None,
                 osd_on="last", warm=False):
    """(W,F) sliding-window decode of whole shots; returns dict(fail, det_out,
    obs_out, win_flags, e (committed correction over DEM columns), edge_iters).
    osd = (bp_iters, lambda, n_keep) decodes the last window (osd_on="all":
    every window) by BP + OSD-CS instead of GDG. warm: each window's
    preprocessing BP starts from the messages the previous window hands over."""
    det = np.ascontiguousarray(det, np.uint8)
    obs = np.ascontiguousarray(obs, np.uint8)
    ns = det.shape[0]
    nwin = n_windows(dem.n_rounds, W, F)
    keep = _dem_args(dem)
    det_out = np.zeros_like(det)
    obs_out = np.zeros_like(obs)
    fail = np.zeros(ns, np.uint8)
    wf = np.zeros((ns, nwin), np.int32)
    ei = np.zeros(1, np.int64)
    e_out = np.zeros((ns, dem.n_cols), np.uint8)
    r = lib().orc_decode_shots(dem.n_rows, dem.n_cols, dem.n_obs, dem.w, dem.n_rounds,
                               *[_p(a) for a in keep], W, C.byref(prm), ns, _p(det), _p(obs),
                               _p(det_out), _p(obs_out), _p(fail), _p(wf), _p(e_out), _p(ei),
                               n_threads or default_threads(), max_windows, F,
                               *(osd if osd else (0, 0, 0)), int(osd_on == "all"), int(warm))
    if r < 0:
        raise ValueError(f"orc_decode_shots failed: {r}")
    return dict(fail=fail, det_out=det_out, obs_out=obs_out, win_flags=wf, e=e_out,
                edge_iters=int(ei[0]))


def select_vn(hist, deg, status, n_unsat, low_error, D, on_main):
    hist = np.ascontiguousarray(hist, np.float64)
    n = hist.shape[0]
    deg = np.ascontiguousarray(deg, np.int32)
    status = np.ascontiguousarray(status, np.int32)
    n_unsat = np.ascontiguousarray(n_unsat, np.int32)
    fav = np.zeros(1, np.int32)
    agg = np.zeros(n, np.int32)
    g = lib().orc_select_vn(n, _p(hist), _p(deg), _p(status), _p(n_unsat), int(low_error), D,
                            int(on_main), _p(fav), _p(agg))
    return g, int(fav[0]), agg


def agg_dec(hist4, D, on_main, n_unsat):
    h = np.ascontiguousarray(hist4, np.float64)
    return lib().orc_agg_dec(_p(h), D, int(on_main), n_unsat)


def path_value(prm, pid, D, f):
    om = np.zeros(1, np.int32)
    dm = np.zeros(1, np.int32)
    v = lib().orc_path_value(C.byref(prm), pid, D, f, _p(om), _p(dm))
    return v, bool(om[0]), int(dm[0])


def n_paths(prm):
    return lib().orc_n_paths(C.byref(prm))


def peel(H, status, s):
    H = np.ascontiguousarray(H, np.uint8)
    st = np.ascontiguousarray(status, np.int32).copy()
    ss = np.ascontiguousarray(s, np.int32).copy()
    ok = lib().orc_peel(H.shape[0], H.shape[1], _p(H), _p(st), _p(ss))
    return bool(ok), st, ss


def dense_bp(H, llr, syn, prm, n_iters):
    H = np.ascontiguousarray(H, np.uint8)
    llr = np.ascontiguousarray(llr, np.float64)
    syn = np.ascontiguousarray(syn, np.uint8)
    post = np.zeros((n_iters, H.shape[1]), np.float64)
    lib().orc_dense_bp(H.shape[0], H.shape[1], _p(H), _p(llr), _p(syn), C.byref(prm), n_iters,
                       _p(post))
    return post


def dense_gdg(H, llr, syn, prm):
    H = np.ascontiguousarray(H, np.uint8)
    llr = np.ascontiguousarray(llr, np.float64)
    syn = np.ascontiguousarray(syn, np.uint8)
    e = np.zeros(H.shape[1], np.uint8)
    fl = np.zeros(1, np.int32)
    pm = lib().orc_dense_gdg(H.shape[0], H.shape[1], _p(H), _p(llr), _p(syn), C.byref(prm),
                             _p(e), _p(fl))
    return pm, e, int(fl[0])


def dense_window(H, llr, syn, prm, warm_in=None, warm_out=False):
    """decode_window on a dense problem (preprocessing, ranking and truncation
    included when prm.pre_iters > 0). Returns dict(pm, e, flags, kept (ranked
    kept columns), lsum (ranking keys)). warm_in: CN-to-VN messages per edge
    (row-major, NaN: none) the preprocessing BP starts from; warm_out=True adds
    the messages the window hands over ("warm_out")."""
    H = np.ascontiguousarray(H, np.uint8)
    llr = np.ascontiguousarray(llr, np.float64)
    syn = np.ascontiguousarray(syn, np.uint8)
    n = H.shape[1]
    ne = int(H.sum())
    e = np.zeros(n, np.uint8)
    fl = np.zeros(1, np.int32)
    kept = np.full(n, -1, np.int32)
    nk = np.zeros(1, np.int32)
    lsum = np.zeros(n, np.float64)
    wi = None if warm_in is None else np.ascontiguousarray(warm_in, np.float64)
    wo = np.zeros(ne, np.float64) if warm_out else None
    pm = lib().orc_dense_window(H.shape[0], n, _p(H), _p(llr), _p(syn), C.byref(prm), _p(e),
                                _p(fl), _p(kept), _p(nk), _p(lsum), _p(wi), _p(wo))
    out = dict(pm=pm, e=e, flags=int(fl[0]), kept=kept[:int(nk[0])], lsum=lsum)
    if warm_out:
        out["warm_out"] = wo
    return out


def dense_path_probe(H, llr, syn, prm, path_id=0, max_steps=8):
    """One GDG path on a dense problem (no preprocessing) with per-step
    diagnostics: posteriors and history at the end of each step's BP run, the
    status before the Alg. 3 pass, unsatisfied-CN counts and Alg. 3 decisions."""
    H = np.ascontiguousarray(H, np.uint8)
    llr = np.ascontiguousarray(llr, np.float64)
    syn = np.ascontiguousarray(syn, np.uint8)
    n = H.shape[1]
    f = lambda: np.full((max_steps, n), np.nan)
    i = lambda: np.full((max_steps, n), -9, np.int32)
    post, hsum, hmin, hmax = f(), f(), f(), f()
    status, nu, agg = i(), i(), i()
    steps = lib().orc_dense_path_probe(H.shape[0], n, _p(H), _p(llr), _p(syn), C.byref(prm),
                                       path_id, max_steps, _p(post), _p(hsum), _p(hmin),
                                       _p(hmax), _p(status), _p(nu), _p(agg))
    k = max(steps, 0)
    return dict(steps=steps, post=post[:k], hsum=hsum[:k], hmin=hmin[:k], hmax=hmax[:k],
                status=status[:k], n_unsat=nu[:k], agg=agg[:k])


def dense_osd(H, llr, syn, prm, n_iters=0, cs=True, lam=10, n_keep=0):
    """BP + OSD-CS on a dense problem (n_iters = 0: OSD on the priors)."""
    H = np.ascontiguousarray(H, np.uint8)
    llr = np.ascontiguousarray(llr, np.float64)
    syn = np.ascontiguousarray(syn, np.uint8)
    e = np.zeros(H.shape[1], np.uint8)
    fl = np.zeros(1, np.int32)
    pm = lib().orc_dense_osd(H.shape[0], H.shape[1], _p(H), _p(llr), _p(syn), C.byref(prm),
                             n_iters, int(cs), lam, n_keep, _p(e), _p(fl))
    return pm, e, int(fl[0])
