"""Learned decimation proposer: training data, training, and decoding.

The proposer is this project's addition to GDG (the paper selects with
Alg. 1). At every decimation step it scores the first 16 candidates in
Alg. 1's order -- features: a candidate's last 16 BP posteriors, squashed
as p / (8 + |p|), and its degree / 8 -- with a 17-64-64-1 network whose
output is the logit that the candidate is in error, and decimates the
candidate most likely in error to the network's decision. The learned paths
guess either at depths 1..g as in Fig. 2 (the default, g = 2: 4 paths) or at
the steps where the decision is not confident. Plain GDG decodes any window
the learned paths cannot satisfy, so every committed correction still meets
its window syndrome when plain GDG's would.

Training data comes from the project's own sampler: shots at noise levels p
drawn from a range, decoded with plain GDG in record mode on one of their
windows (the earlier ones decoded and committed first); each recorded
candidate is labelled with the sampled error bit of its DEM column, or for a
unit column with the parity of the merged columns' errors on its row. The network is trained on the GPU with the library's FP32
forward/backward kernels and Adam.
"""
from __future__ import annotations

import os

import numpy as np
import torch

from . import gdg as G

HERE = os.path.dirname(os.path.abspath(__file__))
N_CAND = 16


def init_params(seed: int) -> torch.Tensor:
    """He-scaled initial parameters on the device (FP32)."""
    rng = np.random.default_rng(seed)
    i, h = G.MLP_IN, G.MLP_H
    w1 = rng.normal(0, np.sqrt(2.0 / i), (i, h))
    w2 = rng.normal(0, np.sqrt(2.0 / h), (h, h))
    w3 = rng.normal(0, np.sqrt(1.0 / h), h)
    p = np.concatenate([w1.ravel(), np.zeros(h), w2.ravel(), np.zeros(h), w3, [0.0]])
    return torch.from_numpy(p.astype(np.float32)).cuda()


def unit_column_sources(dem, src: np.ndarray, row0: int) -> dict:
    """For each unit column of a window (the columns reaching past its last
    round, merged per last-round row they touch; Sec. III), the DEM columns
    merged into it: those touching that row that start inside the window and
    are not window columns themselves. src: the window's column table (DEM
    column, or -1 - local row for a unit column); row0: its first DEM row.
    Keyed by the unit column's local row."""
    src = np.asarray(src)
    own = np.zeros(dem.n_cols, bool)
    own[src[src >= 0]] = True
    first = dem.first_round()
    k_round = row0 // dem.w
    edge_col = np.repeat(np.arange(dem.n_cols), np.diff(np.asarray(dem.h_ptr)))
    edge_row = np.asarray(dem.h_idx)
    keep = ~own[edge_col] & (first[edge_col] >= k_round)
    out = {}
    for r in (-1 - src[src < 0]).tolist():
        out[r] = np.unique(edge_col[keep & (edge_row == row0 + r)]).astype(np.int64)
    return out


def record(dem, prm: G.Params, n_shots: int, seed: int, stream: int = 0, rec_steps: int = 8,
           chunk: int = 20000, window: int = 0):
    """Features x [N, 17] and labels y [N] (float 0/1) of the candidates met on
    the plain main path of window `window` of n_shots sampled shots (the
    earlier windows decoded with plain GDG and committed first). A candidate's
    label is the sampled error bit of its DEM column; for a unit column, the
    parity of the errors of the columns merged into it on its row (Alg. 1
    offers only VNs of degree 3 or more and unit columns have degree 1, so
    this case arises only if candidates are ever drawn more widely)."""
    dev = torch.device("cuda")
    wins = [G.Window(dem, k, 3, prm) for k in range(window + 1)]
    win = wins[window]
    src_np = win.columns()[0].astype(np.int64)
    src = torch.from_numpy(src_np).to(dev)
    units = unit_column_sources(dem, src_np, win.row0) if (src_np < 0).any() else {}
    ddem = G.DeviceDem(dem)
    work = G.learned_work(win)
    xs, ys = [], []
    for s0 in range(0, n_shots, chunk):
        n = min(chunk, n_shots - s0)
        det, obs = ddem.sample(n, seed=seed, stream=stream, shot0=s0, device=dev)
        err = G.sample_errors(ddem, n, seed=seed, stream=stream, shot0=s0, device=dev)
        for w in wins[:window]:
            eh, _, _ = w.decode(det, syn_offset=w.row0)
            w.commit(eh, det, obs)
        # unit-column truth per local row: parity of the merged columns' errors
        unit_truth = torch.zeros((n, win.m), dtype=torch.int32, device=dev)
        for r, cols in units.items():
            if cols.size:
                unit_truth[:, r] = err[:, torch.from_numpy(cols).to(dev)].int().sum(1) % 2
        rx = torch.zeros((n, rec_steps, N_CAND, G.MLP_IN), dtype=torch.float32, device=dev)
        rc = torch.full((n, rec_steps, N_CAND), -1, dtype=torch.int32, device=dev)
        rf = torch.zeros((n, rec_steps, N_CAND), dtype=torch.int32, device=dev)
        cfg = G.LearnCfg(2, N_CAND, 0, 0.0, rec_steps, rx.data_ptr(), rc.data_ptr(),
                         rf.data_ptr(), None, float("inf"))
        G.decode_learned(win, det, win.row0, cfg, work=work)
        ok = rc >= 0
        shot = torch.arange(n, device=dev).view(n, 1, 1).expand_as(rc)[ok]
        dcol = src[rc[ok].long()]
        col_truth = err[shot, dcol.clamp(min=0)].int()
        row_truth = unit_truth[shot, (-1 - dcol).clamp(min=0)]
        truth = torch.where(dcol >= 0, col_truth, row_truth)
        xs.append(rx[ok])
        ys.append(truth.float())
    return torch.cat(xs), torch.cat(ys)


def train(x: torch.Tensor, y: torch.Tensor, epochs: int = 3, batch: int = 8192, lr: float = 2e-3,
          seed: int = 0, log=None) -> torch.Tensor:
    """Adam on the mean binary cross-entropy; returns the FP32 parameters."""
    params = init_params(seed)
    tr = G.MlpTrainer(params, batch)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    n = x.shape[0]
    for ep in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=gen)
        tot, nb = 0.0, 0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            loss = tr.step(x[idx].contiguous(), y[idx].contiguous(), lr=lr * (0.5 ** ep))
            if nb % 50 == 0:
                tot += float(loss.item())
            nb += 1
        if log:
            log(f"epoch {ep}: {nb} steps, sampled mean loss {tot / max(1, (nb + 49) // 50):.4f}")
    return params


def save(params: torch.Tensor, path: str):
    np.save(path, params.detach().cpu().numpy().astype(np.float32), allow_pickle=False)


def load(path: str) -> np.ndarray:
    p = np.load(path, allow_pickle=False)
    if p.shape != (G.MLP_PARAMS,):
        raise ValueError(f"{path}: expected {G.MLP_PARAMS} parameters")
    return p


def default_model_path(code_key: str = "144") -> str:
    return os.path.join(HERE, f"proposer_{code_key}.npy")


class LearnedSlidingWindowDecoder:
    """(W,1) sliding window as SlidingWindowDecoder, each window decoded by the
    learned paths with plain GDG as fallback."""

    def __init__(self, dem, prm: G.Params, params, W: int = 3, guesses: int = 2,
                 tau: float = 1.0, n_cand: int = N_CAND, pm_fallback: float = float("inf"),
                 tree: bool = True):
        self.dem = dem
        self.W = W
        self.n_windows = dem.n_rounds - W + 1
        self.windows = [G.Window(dem, k, W, prm) for k in range(self.n_windows)]
        self.model = G.Model(params)
        self.guesses, self.tau, self.n_cand = guesses, tau, n_cand
        self.pm_fallback = pm_fallback
        self.tree = tree
        self.work = G.learned_work(self.windows[0])
        for w in self.windows[1:]:
            if G.lib().gdg_learned_work_bytes(w.h) > self.work.numel():
                self.work = G.learned_work(w)

    def cfg(self, edge_iters=None):
        return G.LearnCfg(1, self.n_cand, self.guesses, self.tau, 0, None, None, None,
                          edge_iters.data_ptr() if edge_iters is not None else None,
                          self.pm_fallback, int(self.tree))

    def decode(self, det: torch.Tensor, obs: torch.Tensor, edge_iters: torch.Tensor = None):
        """In place like SlidingWindowDecoder.decode; returns (fail, window flags).
        edge_iters [n_shots, n_windows] (int64, optional) receives the BP work."""
        ns = det.shape[0]
        wflags = torch.empty((ns, self.n_windows), dtype=torch.int32, device=det.device)
        for k, w in enumerate(self.windows):
            ei = None
            if edge_iters is not None:
                ei = torch.empty(ns, dtype=torch.int64, device=det.device)
            ehat, pm, fl = G.decode_learned(w, det, w.row0, self.cfg(ei), self.model, self.work)
            if ei is not None:
                edge_iters[:, k] = ei
            wflags[:, k] = fl
            w.commit(ehat, det, obs)
        return G.evaluate(det, obs), wflags
