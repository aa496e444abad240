"""Python binding of the gdg C ABI (include/gdg.h): argument marshalling only.

Every step of the decoder runs in the HIP library libgdg_hip.so; torch supplies
device memory and the current stream. If the library is missing the calls
raise -- there is no other implementation to fall back to.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgdg_hip.so")

GDG_FLAG_SATISFIED = 1
GDG_FLAG_CONTRADICTION = 2
GDG_FLAG_EXHAUSTED = 4
GDG_FLAG_FALLBACK = 8
GDG_FLAG_CAPACITY = 16

EXPORTED = ["gdg_build_window", "gdg_window_free", "gdg_window_get_info", "gdg_window_columns",
            "gdg_workspace_bytes", "gdg_decode_batch", "gdg_decode_jobs", "gdg_jobs_lds_bytes",
            "gdg_commit", "gdg_commit_indexed", "gdg_copy_rows", "gdg_bp", "gdg_dem_upload",
            "gdg_dem_free", "gdg_sample", "gdg_sample_errors", "gdg_evaluate",
            "gdg_mlp_forward", "gdg_mlp_grad_work_bytes", "gdg_mlp_grad", "gdg_mlp_adam",
            "gdg_model_create", "gdg_model_free", "gdg_mlp_infer", "gdg_learned_work_bytes",
            "gdg_decode_learned", "gdg_last_error", "gdg_decode_batch_noalloc",
            "gdg_release_scratch", "gdg_decode_osd", "gdg_link_windows", "gdg_window_edge_slots",
            "gdg_decode_batch_warm", "gdg_decode_chain"]

MLP_IN, MLP_H = 17, 64
MLP_PARAMS = 5377


class Dem(C.Structure):
    _fields_ = [("n_rows", C.c_int32), ("n_cols", C.c_int32), ("n_obs", C.c_int32),
                ("w", C.c_int32), ("n_rounds", C.c_int32), ("h_ptr", C.c_void_p),
                ("h_idx", C.c_void_p), ("l_ptr", C.c_void_p), ("l_idx", C.c_void_p),
                ("priors", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("alpha", C.c_float), ("clip", C.c_float), ("iters_per_step", C.c_int32),
                ("pre_iters", C.c_int32), ("trunc_factor", C.c_int32), ("g", C.c_int32),
                ("dmax_main", C.c_int32), ("extra_steps", C.c_int32),
                ("side_max_depth", C.c_int32), ("low_error", C.c_int32)]


class WindowInfo(C.Structure):
    _fields_ = [(f, C.c_int32) for f in ("k", "W", "m", "n", "row0", "n_act", "n_paths", "n_edges",
                                         "max_sub_edges", "n_commit", "last", "lds_bytes",
                                         "waves", "n_msg")]


class Trace(C.Structure):
    _fields_ = [("sel", C.c_void_p), ("dec", C.c_void_p), ("log_cap", C.c_int32),
                ("ends", C.c_void_p), ("first_post", C.c_void_p), ("edge_iters", C.c_void_p),
                ("step_lsum", C.c_void_p), ("pre_post", C.c_void_p)]


class Job(C.Structure):
    _fields_ = [("win", C.c_void_p), ("n_shots", C.c_int32), ("d_syndrome", C.c_void_p),
                ("syn_stride", C.c_int64), ("d_ehat", C.c_void_p), ("d_pm", C.c_void_p),
                ("d_flags", C.c_void_p)]


class LaunchCfg(C.Structure):
    _fields_ = [("waves", C.c_int32), ("workgroups", C.c_int32)]


class LearnCfg(C.Structure):
    _fields_ = [("mode", C.c_int32), ("n_cand", C.c_int32), ("guesses", C.c_int32),
                ("tau", C.c_float), ("rec_steps", C.c_int32), ("d_rec_x", C.c_void_p),
                ("d_rec_col", C.c_void_p), ("d_rec_fav", C.c_void_p),
                ("d_edge_iters", C.c_void_p), ("pm_fallback", C.c_float), ("tree", C.c_int32)]


MAX_JOBS = 8


def params(alpha=1.0, clip=50.0, iters_per_step=6, pre_iters=0, trunc_factor=2, g=0,
           dmax_main=25, extra_steps=10, side_max_depth=0, low_error=1) -> Params:
    return Params(alpha, clip, iters_per_step, pre_iters, trunc_factor, g, dmax_main,
                  extra_steps, side_max_depth, low_error)


def paper_params(n_qubits: int, p: float, **over) -> Params:
    """The decoder settings the paper uses for an N-qubit BB code under
    circuit-level noise (Sec. IV-C, Fig. 2): for N <= 144 a depth-4 guessing
    tree with side paths splitting up to depth 10 (22 paths), main D_max 25,
    10 steps after a split, 8 preprocessing iterations; for N = 288 a depth-5
    tree, side paths up to depth 20 (47 paths), main D_max 40, 20 steps after
    a split, 16 preprocessing iterations. Low-error mode (no Alg. 3) for
    p <= 0.002 (Sec. IV-A). Keyword arguments override fields."""
    if n_qubits >= 288:
        d = dict(g=5, side_max_depth=20, dmax_main=40, extra_steps=20, pre_iters=16)
    else:
        d = dict(g=4, side_max_depth=10, dmax_main=25, extra_steps=10, pre_iters=8)
    d.update(alpha=1.0, trunc_factor=2, low_error=int(p <= 0.002))
    d.update(over)
    return params(**d)


def appendix_params(**over) -> Params:
    """The GDG settings of the one-round problems (App. A data-qubit noise,
    App. B single-shot syndrome noise): low-error mode, main D_max 40, side
    paths splitting up to depth 20, a depth-5 guessing tree, 30 more steps
    after a split, scaling 0.625, and no preprocessing or truncation (the
    window is the whole one-round matrix). Keyword arguments override fields."""
    d = dict(g=5, side_max_depth=20, dmax_main=40, extra_steps=30, alpha=0.625, pre_iters=0,
             low_error=1)
    d.update(over)
    return params(**d)


_lib = None


def lib():
    """Loads libgdg_hip.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2403_18901_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        P, i32, i64, u32, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64
        L.gdg_build_window.argtypes = [P, i32, i32, i32, P, P]
        L.gdg_window_free.argtypes = [P]
        L.gdg_window_get_info.argtypes = [P, P]
        L.gdg_window_columns.argtypes = [P, P, P, P]
        L.gdg_workspace_bytes.argtypes = [P, i32]
        L.gdg_workspace_bytes.restype = C.c_size_t
        L.gdg_decode_batch.argtypes = [P, i32, P, i64, P, P, P, P, C.c_size_t, P, P]
        L.gdg_decode_batch_noalloc.argtypes = [P, i32, P, i64, P, P, P, P]
        L.gdg_release_scratch.argtypes = [P]
        L.gdg_decode_osd.argtypes = [P, i32, P, i64, i32, i32, i32, i32, P, P, P, P, P, P]
        L.gdg_link_windows.argtypes = [P, P]
        L.gdg_decode_chain.argtypes = [P, P, P, i32, i32, P, P, P, P, P, P, P, i64, P, P, P]
        L.gdg_window_edge_slots.argtypes = [P, P]
        L.gdg_decode_batch_warm.argtypes = [P, i32, P, i64, P, i64, P, i64, P, P, P, P,
                                            C.c_size_t, P, P]
        L.gdg_decode_jobs.argtypes = [P, i32, P, P]
        L.gdg_jobs_lds_bytes.argtypes = [P, i32, i32]
        L.gdg_commit.argtypes = [P, i32, P, P, i64, P, i64, P]
        L.gdg_commit_indexed.argtypes = [P, i32, P, P, P, P, P, P]
        L.gdg_copy_rows.argtypes = [i32, i32, P, P, P, P, P]
        L.gdg_bp.argtypes = [P, i32, P, i64, i32, P, P, P]
        L.gdg_dem_upload.argtypes = [P, P]
        L.gdg_dem_free.argtypes = [P]
        L.gdg_sample.argtypes = [P, i32, u64, u32, u64, P, P, P]
        L.gdg_evaluate.argtypes = [i32, i32, i32, P, P, P, P]
        L.gdg_sample_errors.argtypes = [P, i32, u64, u32, u64, P, P]
        L.gdg_mlp_forward.argtypes = [i32, P, P, P, P]
        L.gdg_mlp_grad_work_bytes.argtypes = [i32]
        L.gdg_mlp_grad_work_bytes.restype = C.c_size_t
        L.gdg_mlp_grad.argtypes = [i32, P, P, P, P, P, P, C.c_size_t, P]
        L.gdg_mlp_adam.argtypes = [i32, C.c_float, C.c_float, C.c_float, C.c_float, P, P, P, P, P]
        L.gdg_model_create.argtypes = [P, P]
        L.gdg_model_free.argtypes = [P]
        L.gdg_mlp_infer.argtypes = [P, i32, P, P, P]
        L.gdg_learned_work_bytes.argtypes = [P]
        L.gdg_learned_work_bytes.restype = C.c_size_t
        L.gdg_decode_learned.argtypes = [P, P, P, i32, P, i64, P, P, P, P, C.c_size_t, P]
        L.gdg_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def release_scratch():
    """Frees the library's decode scratch pool of the current stream."""
    _check(lib().gdg_release_scratch(_stream()))


def _check(rc):
    if rc != 0:
        raise RuntimeError(f"gdg error {rc}: {lib().gdg_last_error().decode()}")


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, offset=0):
    return C.c_void_p(t.data_ptr() + offset) if t is not None else None


class _HostDem:
    """Keeps contiguous host arrays alive for a gdg_dem struct."""

    def __init__(self, dem):
        self.arrs = [np.ascontiguousarray(dem.h_ptr, np.int32),
                     np.ascontiguousarray(dem.h_idx, np.int32),
                     np.ascontiguousarray(dem.l_ptr, np.int32),
                     np.ascontiguousarray(dem.l_idx, np.int32),
                     np.ascontiguousarray(dem.priors, np.float64)]
        p = [a.ctypes.data_as(C.c_void_p) for a in self.arrs]
        self.s = Dem(dem.n_rows, dem.n_cols, dem.n_obs, dem.w, dem.n_rounds, *p)


def n_windows(n_rounds: int, W: int, F: int = 1) -> int:
    """Windows of a (W,F) sliding window over n_rounds detector rounds."""
    return 1 if n_rounds <= W else 1 + (n_rounds - W + F - 1) // F


class Window:
    """One window of a (W,F) sliding window, built and held by the library."""

    def __init__(self, dem, k: int, W: int, prm: Params, F: int = 1):
        hd = _HostDem(dem)
        h = C.c_void_p()
        _check(lib().gdg_build_window(C.byref(hd.s), k, W, F, C.byref(prm), C.byref(h)))
        self.h = h
        self.prm = prm
        info = WindowInfo()
        _check(lib().gdg_window_get_info(self.h, C.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in WindowInfo._fields_}
        self.m, self.n, self.row0 = info.m, info.n, info.row0
        self.n_act, self.n_paths = info.n_act, info.n_paths
        self.n_msg, self.n_edges = info.n_msg, info.n_edges
        self.linked = None

    def link(self, prev: "Window"):
        """gdg_link_windows: this window's preprocessing BP may start from the
        messages `prev` hands over (warm start)."""
        _check(lib().gdg_link_windows(self.h, prev.h))
        self.linked = prev   # keeps prev's graph alive while linked

    def edge_slots(self):
        """Message slot of every window edge (row-major CSR) in the warm buffers."""
        slot = np.zeros(self.n_edges, np.int32)
        _check(lib().gdg_window_edge_slots(self.h, slot.ctypes.data_as(C.c_void_p)))
        return slot

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.gdg_window_free(self.h)
            self.h = None

    def columns(self):
        src = np.zeros(self.n, np.int32)
        llr = np.zeros(self.n, np.float64)
        commit = np.zeros(self.n, np.uint8)
        _check(lib().gdg_window_columns(self.h, src.ctypes.data_as(C.c_void_p),
                                        llr.ctypes.data_as(C.c_void_p),
                                        commit.ctypes.data_as(C.c_void_p)))
        return src, llr, commit

    def decode(self, syn: torch.Tensor, syn_offset: int = 0, n_shots: int | None = None,
               trace: bool = False, log_cap: int = 32, out=None, step_lsum: bool = False,
               pre_post: bool = False, warm_in: torch.Tensor | None = None,
               warm_out: torch.Tensor | None = None):
        """syn: uint8 cuda tensor [n_shots, stride]; window rows start at column syn_offset.
        warm_in / warm_out: float32 cuda tensors [n_shots, >= n_msg] of handed-over
        messages (gdg_decode_batch_warm); warm_in needs link()."""
        assert syn.dtype == torch.uint8 and syn.is_cuda and syn.dim() == 2 and syn.is_contiguous()
        ns = syn.shape[0] if n_shots is None else n_shots
        dev = syn.device
        if out is None:
            ehat = torch.empty((ns, self.n), dtype=torch.uint8, device=dev)
            pm = torch.empty(ns, dtype=torch.float64, device=dev)
            flags = torch.empty(ns, dtype=torch.int32, device=dev)
        else:
            ehat, pm, flags = out
        tr = None
        trd = None
        if trace:
            trd = dict(sel=torch.empty((ns, self.n_act), dtype=torch.int32, device=dev),
                       dec=torch.empty((ns, self.n_paths, log_cap, 3), dtype=torch.int32,
                                       device=dev),
                       ends=torch.empty((ns, self.n_paths, 2), dtype=torch.int32, device=dev),
                       first_post=torch.empty((ns, self.n_act), dtype=torch.float32, device=dev),
                       edge_iters=torch.empty(ns, dtype=torch.int64, device=dev))
            if step_lsum:
                trd["step_lsum"] = torch.empty((ns, self.n_paths, log_cap, self.n_act),
                                               dtype=torch.float32, device=dev)
            if pre_post:
                trd["pre_post"] = torch.empty((ns, self.prm.pre_iters, self.n),
                                              dtype=torch.float32, device=dev)
            tr = Trace(_ptr(trd["sel"]), _ptr(trd["dec"]), log_cap, _ptr(trd["ends"]),
                       _ptr(trd["first_post"]), _ptr(trd["edge_iters"]),
                       _ptr(trd.get("step_lsum")), _ptr(trd.get("pre_post")))
        if warm_in is not None or warm_out is not None:
            for t in (warm_in, warm_out):
                assert t is None or (t.dtype == torch.float32 and t.is_cuda and t.dim() == 2
                                     and t.is_contiguous() and t.shape[0] >= ns)
            _check(lib().gdg_decode_batch_warm(
                self.h, ns, _ptr(syn, syn_offset), syn.shape[1], _ptr(warm_in),
                warm_in.shape[1] if warm_in is not None else 0, _ptr(warm_out),
                warm_out.shape[1] if warm_out is not None else 0, _ptr(ehat), _ptr(pm),
                _ptr(flags), None, 0, C.byref(tr) if tr is not None else None, _stream()))
        else:
            _check(lib().gdg_decode_batch(self.h, ns, _ptr(syn, syn_offset), syn.shape[1],
                                          _ptr(ehat), _ptr(pm), _ptr(flags), None, 0,
                                          C.byref(tr) if tr is not None else None, _stream()))
        if trace:
            return ehat, pm, flags, trd
        return ehat, pm, flags

    def workspace_bytes(self, n_shots: int) -> int:
        return int(lib().gdg_workspace_bytes(self.h, n_shots))

    def decode_into(self, syn: torch.Tensor, syn_offset: int, out, workspace=None,
                    noalloc: bool = False, n_shots: int | None = None):
        """gdg_decode_batch into caller buffers out = (ehat, pm, flags), with an
        optional caller workspace (uint8 cuda tensor), or
        gdg_decode_batch_noalloc when noalloc is set."""
        ns = syn.shape[0] if n_shots is None else n_shots
        ehat, pm, flags = out
        if noalloc:
            _check(lib().gdg_decode_batch_noalloc(self.h, ns, _ptr(syn, syn_offset), syn.shape[1],
                                                  _ptr(ehat), _ptr(pm), _ptr(flags), _stream()))
        else:
            _check(lib().gdg_decode_batch(self.h, ns, _ptr(syn, syn_offset), syn.shape[1],
                                          _ptr(ehat), _ptr(pm), _ptr(flags), _ptr(workspace),
                                          workspace.numel() if workspace is not None else 0,
                                          None, _stream()))
        return out

    def decode_osd(self, syn: torch.Tensor, syn_offset: int = 0, bp_iters: int = 200,
                   cs: bool = True, lam: int = 10, n_keep: int = 0, trace: bool = False,
                   out=None):
        """BP + OSD-CS(lam) (OSD-0 with cs=False) on the window (gdg_decode_osd);
        n_keep > 0 keeps the first n_keep ranked columns. Returns (ehat, pm,
        flags) and, with trace, (order, bp_iters) too."""
        ns = syn.shape[0]
        dev = syn.device
        if out is None:
            out = (torch.empty((ns, self.n), dtype=torch.uint8, device=dev),
                   torch.empty(ns, dtype=torch.float64, device=dev),
                   torch.empty(ns, dtype=torch.int32, device=dev))
        ehat, pm, flags = out
        order = it = None
        if trace:
            order = torch.empty((ns, self.n), dtype=torch.int32, device=dev)
            it = torch.empty(ns, dtype=torch.int32, device=dev)
        _check(lib().gdg_decode_osd(self.h, ns, _ptr(syn, syn_offset), syn.shape[1], bp_iters,
                                    int(cs), lam, n_keep, _ptr(ehat), _ptr(pm), _ptr(flags),
                                    _ptr(order), _ptr(it), _stream()))
        if trace:
            return ehat, pm, flags, order, it
        return ehat, pm, flags

    def commit(self, ehat: torch.Tensor, det: torch.Tensor, obs: torch.Tensor):
        ns = ehat.shape[0]
        _check(lib().gdg_commit(self.h, ns, _ptr(ehat), _ptr(det), det.shape[1], _ptr(obs),
                                obs.shape[1] if obs.dim() == 2 else 0, _stream()))

    def commit_indexed(self, ehat: torch.Tensor, det: torch.Tensor, det_off: torch.Tensor,
                       obs: torch.Tensor, obs_off: torch.Tensor):
        """Commit for shots whose window rows start at det_off[i] (int64 element
        offsets into det) and whose observables start at obs_off[i]."""
        ns = ehat.shape[0]
        _check(lib().gdg_commit_indexed(self.h, ns, _ptr(ehat), _ptr(det), _ptr(det_off),
                                        _ptr(obs), _ptr(obs_off), _stream()))

    def bp(self, syn: torch.Tensor, n_iters: int, syn_offset: int = 0):
        ns = syn.shape[0]
        post = torch.empty((ns, n_iters, self.n), dtype=torch.float32, device=syn.device)
        first = torch.empty(ns, dtype=torch.int32, device=syn.device)
        _check(lib().gdg_bp(self.h, ns, _ptr(syn, syn_offset), syn.shape[1], n_iters, _ptr(post),
                            _ptr(first), _stream()))
        return post, first


def decode_jobs(jobs, waves: int = 4, workgroups: int = 0):
    """One persistent launch over several (window, syndromes, outputs) jobs.

    jobs: list of (Window, syn tensor [n_shots, stride] uint8, syn_offset,
    (ehat, pm, flags)) with ehat [n_shots, window.n] uint8, pm [n_shots] f64,
    flags [n_shots] i32. Order matters for load balance: costliest first.
    """
    if not 1 <= len(jobs) <= MAX_JOBS:
        raise ValueError(f"1..{MAX_JOBS} jobs per launch")
    arr = (Job * len(jobs))()
    for i, (w, syn, off, (ehat, pm, fl)) in enumerate(jobs):
        assert syn.dtype == torch.uint8 and syn.is_contiguous() and ehat.shape[1] == w.n
        arr[i] = Job(w.h, syn.shape[0], _ptr(syn, off), syn.shape[1], _ptr(ehat), _ptr(pm),
                     _ptr(fl))
    cfg = LaunchCfg(waves, workgroups)
    _check(lib().gdg_decode_jobs(C.cast(arr, C.c_void_p), len(jobs), C.byref(cfg), _stream()))


def jobs_lds_bytes(windows, waves: int) -> int:
    arr = (Job * len(windows))()
    for i, w in enumerate(windows):
        arr[i] = Job(w.h, 0, None, w.m, None, None, None)
    return lib().gdg_jobs_lds_bytes(C.cast(arr, C.c_void_p), len(windows), waves)


class DeviceDem:
    """Device copy of a DEM for sampling shots on the GPU."""

    def __init__(self, dem):
        hd = _HostDem(dem)
        h = C.c_void_p()
        _check(lib().gdg_dem_upload(C.byref(hd.s), C.byref(h)))
        self.h = h
        self.n_rows, self.n_obs, self.n_cols = dem.n_rows, dem.n_obs, dem.n_cols

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.gdg_dem_free(self.h)
            self.h = None

    def sample(self, n_shots: int, seed: int, stream: int = 0, shot0: int = 0, device="cuda",
               out=None):
        if out is None:
            det = torch.empty((n_shots, self.n_rows), dtype=torch.uint8, device=device)
            obs = torch.empty((n_shots, max(self.n_obs, 1)), dtype=torch.uint8, device=device)
        else:
            det, obs = out
        _check(lib().gdg_sample(self.h, n_shots, seed, stream, shot0, _ptr(det), _ptr(obs),
                                _stream()))
        return det, obs


def decode_chain(first: Window, middle, last, n_windows: int, k_begin: torch.Tensor,
                 k_end: torch.Tensor, det: torch.Tensor, det_off: torch.Tensor,
                 obs: torch.Tensor, obs_off: torch.Tensor, ehat: torch.Tensor, pm: torch.Tensor,
                 flags: torch.Tensor):
    """gdg_decode_chain: item i decodes and commits windows k_begin[i] ..
    k_end[i]-1 of the record at flat element offset det_off[i] of det (and the
    observables at obs_off[i] of obs) in one launch. k_begin/k_end int32,
    offsets int64, ehat uint8 [items, >= largest n], pm float64 and flags int32
    [items, n_windows]."""
    n = k_begin.shape[0]
    assert ehat.dim() == 2 and ehat.shape[0] >= n and pm.shape[1] == n_windows
    _check(lib().gdg_decode_chain(first.h, middle.h if middle is not None else None,
                                  last.h if last is not None else None, n_windows, n,
                                  _ptr(k_begin), _ptr(k_end), _ptr(det), _ptr(det_off), _ptr(obs),
                                  _ptr(obs_off), _ptr(ehat), ehat.shape[1], _ptr(pm), _ptr(flags),
                                  _stream()))


def copy_rows(src: torch.Tensor, src_off: torch.Tensor, m: int, dst: torch.Tensor,
              dst_off: torch.Tensor = None):
    """dst[dst_off[i] + j] = src[src_off[i] + j] for j < m (flat uint8 element
    offsets, int64 on the device); dst_off None: row i of a [n, m] dst."""
    n = src_off.shape[0]
    _check(lib().gdg_copy_rows(n, m, _ptr(src), _ptr(src_off), _ptr(dst), _ptr(dst_off),
                               _stream()))
    return dst


def evaluate(det: torch.Tensor, obs: torch.Tensor, out=None) -> torch.Tensor:
    ns = det.shape[0]
    fail = out if out is not None else torch.empty(ns, dtype=torch.uint8, device=det.device)
    _check(lib().gdg_evaluate(ns, det.shape[1], obs.shape[1], _ptr(det), _ptr(obs), _ptr(fail),
                              _stream()))
    return fail


class SlidingWindowDecoder:
    """(W,F) sliding-window GDG over a DEM: window k is decoded on the current
    residual detectors and committed before window k+1 (Sec. III; F > 1 in
    App. E)."""

    def __init__(self, dem, prm: Params, W: int = 3, F: int = 1, osd=None,
                 osd_on: str = "last", warm: bool = False):
        """osd = (bp_iters, lambda, n_keep): the last window (osd_on="all":
        every window) is decoded by BP + OSD-CS instead of GDG (Sec. III's
        window comparator; App. E's last-window variant). warm: each window's
        preprocessing BP starts from the messages the previous one hands over
        (Sec. V's message reuse, gdg_decode_batch_warm)."""
        if osd_on not in ("last", "all"):
            raise ValueError("osd_on is 'last' or 'all'")
        self.dem = dem
        self.W, self.F = W, F
        self.osd, self.osd_on = osd, osd_on
        self.n_windows = n_windows(dem.n_rounds, W, F)
        self.windows = [Window(dem, k, W, prm, F) for k in range(self.n_windows)]
        self.warm = warm and prm.pre_iters > 0
        if self.warm:
            for k in range(1, self.n_windows):
                self.windows[k].link(self.windows[k - 1])

    def decode(self, det: torch.Tensor, obs: torch.Tensor, trace: bool = False):
        """Decodes in place: det becomes the residual detector record and obs the
        observable accumulator (true observables XOR L e). Returns per-shot
        failure flags (Eq. 8 and Eq. 9) and per-window flags."""
        ns = det.shape[0]
        wflags = torch.empty((ns, self.n_windows), dtype=torch.int32, device=det.device)
        traces = []
        bufs = [None, None]
        if self.warm:
            slots = max(w.n_msg for w in self.windows)
            bufs = [torch.empty((ns, slots), dtype=torch.float32, device=det.device)
                    for _ in range(2)]
        carried = False
        for k, w in enumerate(self.windows):
            if self.osd and (self.osd_on == "all" or k == self.n_windows - 1):
                it, lam, keep = self.osd
                res = w.decode_osd(det, syn_offset=w.row0, bp_iters=it, cs=True, lam=lam,
                                   n_keep=keep)
                carried = False
            elif self.warm:
                res = w.decode(det, syn_offset=w.row0, trace=trace,
                               warm_in=bufs[(k + 1) % 2] if carried else None,
                               warm_out=bufs[k % 2] if k + 1 < self.n_windows else None)
                carried = True
            else:
                res = w.decode(det, syn_offset=w.row0, trace=trace)
            ehat, pm, fl = res[:3]
            if trace:
                traces.append(res[3] if len(res) > 3 else None)
            wflags[:, k] = fl
            w.commit(ehat, det, obs)
        fail = evaluate(det, obs)
        if trace:
            return fail, wflags, traces
        return fail, wflags


# ------------------------------------------------------------------ learned proposer

def mlp_forward(params: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """FP32 logits of the proposer network for features x [n, 17]."""
    n = x.shape[0]
    z = torch.empty(n, dtype=torch.float32, device=x.device)
    _check(lib().gdg_mlp_forward(n, _ptr(params), _ptr(x), _ptr(z), _stream()))
    return z


class MlpTrainer:
    """Buffers for gradient steps of the proposer network on the device."""

    def __init__(self, params: torch.Tensor, max_batch: int):
        self.params = params
        self.grad = torch.zeros_like(params)
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=params.device)
        nb = lib().gdg_mlp_grad_work_bytes(max_batch)
        self.work = torch.empty(max(nb, 4), dtype=torch.uint8, device=params.device)
        self.max_batch = max_batch
        self.t = 0

    def gradient(self, x: torch.Tensor, y: torch.Tensor):
        n = x.shape[0]
        if n > self.max_batch:
            raise ValueError("batch larger than the trainer's workspace")
        _check(lib().gdg_mlp_grad(n, _ptr(self.params), _ptr(x), _ptr(y), _ptr(self.grad),
                                  _ptr(self.loss), _ptr(self.work), self.work.numel(), _stream()))
        return self.grad, self.loss

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        _check(lib().gdg_mlp_adam(self.t, lr, b1, b2, eps, _ptr(self.params), _ptr(self.grad),
                                  _ptr(self.m), _ptr(self.v), _stream()))

    def step(self, x, y, lr=1e-3):
        self.gradient(x, y)
        self.adam(lr)
        return self.loss


class Model:
    """Device inference copy (BF16 weights) of FP32 proposer parameters."""

    def __init__(self, params):
        p = np.ascontiguousarray(
            params.detach().float().cpu().numpy() if isinstance(params, torch.Tensor) else params,
            np.float32)
        if p.size != MLP_PARAMS:
            raise ValueError(f"expected {MLP_PARAMS} parameters")
        h = C.c_void_p()
        _check(lib().gdg_model_create(p.ctypes.data_as(C.c_void_p), C.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.gdg_model_free(self.h)
            self.h = None

    def infer(self, x: torch.Tensor) -> torch.Tensor:
        n = x.shape[0]
        z = torch.empty(n, dtype=torch.float32, device=x.device)
        _check(lib().gdg_mlp_infer(self.h, n, _ptr(x), _ptr(z), _stream()))
        return z


def sample_errors(ddem: "DeviceDem", n_shots: int, seed: int, stream: int = 0, shot0: int = 0,
                  device="cuda") -> torch.Tensor:
    err = torch.empty((n_shots, ddem.n_cols), dtype=torch.uint8, device=device)
    _check(lib().gdg_sample_errors(ddem.h, n_shots, seed, stream, shot0, _ptr(err), _stream()))
    return err


def learned_work(win: "Window") -> torch.Tensor:
    nb = lib().gdg_learned_work_bytes(win.h)
    return torch.empty(nb, dtype=torch.uint8, device="cuda")


def decode_learned(win: "Window", syn: torch.Tensor, syn_offset: int, cfg: LearnCfg, model=None,
                   work=None, out=None):
    """Mode 1 or 2 decode of one window (see gdg_decode_learned)."""
    ns = syn.shape[0]
    dev = syn.device
    if out is None:
        out = (torch.empty((ns, win.n), dtype=torch.uint8, device=dev),
               torch.empty(ns, dtype=torch.float64, device=dev),
               torch.empty(ns, dtype=torch.int32, device=dev))
    if work is None:
        work = learned_work(win)
    ehat, pm, fl = out
    _check(lib().gdg_decode_learned(win.h, model.h if model is not None else None, C.byref(cfg),
                                    ns, _ptr(syn, syn_offset), syn.shape[1], _ptr(ehat), _ptr(pm),
                                    _ptr(fl), _ptr(work), work.numel(), _stream()))
    return out

