"""Detector error models (DEMs): the circuit-code parity-check matrix H_circ,
per-column priors and the logical observable matrix L.

Input generation only (it stands in for the circuit simulator the paper used);
none of the decoder's arithmetic lives here.

Models:

* ``phenomenological_dem`` -- i.i.d. data flips before every noisy round plus
  i.i.d. measurement flips, then one perfect round. Detectors are XORs of the
  same check in consecutive rounds (Sec. II-B); a data flip triggers one round,
  a measurement flip two consecutive rounds (the degree-two VNs of Sec. II-B).
* ``data_noise_dem``, ``single_shot_dem`` -- one noiseless / one noisy
  syndrome measurement of a BB code's H_X under i.i.d. data flips (the
  appendices on data-qubit noise and single-shot syndrome noise).
* ``circuit_dem`` -- a depth-8 BB syndrome-extraction circuit of our own design
  (the paper's circuit comes from another work and is not reproduced), Z-basis
  memory with R noisy rounds and a final noiseless round computed from a data
  measurement (Appendix D), standard circuit depolarising noise (Sec. II), and
  X-type fault propagation by Pauli frames. Columns with identical detector and
  observable support are merged into one with the independent-XOR prior
  p = p1 + p2 - 2 p1 p2 (the linearised model of Sec. II-B).

Columns are ordered by first detector round, so each window is a contiguous
column range.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

from .bb import BBCode, logical_operators


@dataclass
class DEM:
    """Sparse detector error model.

    h_ptr/h_idx: H_circ in CSC (column c's detectors are h_idx[h_ptr[c]:h_ptr[c+1]],
    ascending). l_ptr/l_idx: L in CSC (observable indices per column).
    det_round[r]: detector round of row r. Rows are ordered by round, w per round.
    """
    name: str
    n_rows: int
    n_cols: int
    n_obs: int
    w: int
    n_rounds: int            # detector rounds (noisy rounds + final)
    h_ptr: np.ndarray
    h_idx: np.ndarray
    l_ptr: np.ndarray
    l_idx: np.ndarray
    priors: np.ndarray       # float64 per column
    det_round: np.ndarray    # int32 per row
    info: dict = field(default_factory=dict)

    def col_rows(self, c):
        return self.h_idx[self.h_ptr[c]:self.h_ptr[c + 1]]

    def col_obs(self, c):
        return self.l_idx[self.l_ptr[c]:self.l_ptr[c + 1]]

    def first_round(self) -> np.ndarray:
        return self.det_round[self.h_idx[self.h_ptr[:-1]]]

    def last_round(self) -> np.ndarray:
        return self.det_round[self.h_idx[self.h_ptr[1:] - 1]]

    def dense_h(self) -> np.ndarray:
        h = np.zeros((self.n_rows, self.n_cols), dtype=np.uint8)
        for c in range(self.n_cols):
            h[self.col_rows(c), c] = 1
        return h

    def dense_l(self) -> np.ndarray:
        lm = np.zeros((self.n_obs, self.n_cols), dtype=np.uint8)
        for c in range(self.n_cols):
            lm[self.col_obs(c), c] = 1
        return lm

    def thresholds(self) -> np.ndarray:
        """uint32 Bernoulli thresholds: a column fires iff its uniform u32 < thr."""
        t = np.floor(self.priors * 4294967296.0)
        return np.clip(t, 0, 4294967295).astype(np.uint32)


def _from_columns(name, cols, obs, priors, w, n_rounds, n_obs, info):
    """cols: list of sorted row arrays; obs: list of sorted obs arrays."""
    first = np.array([c[0] // w for c in cols])
    order = np.argsort(first, kind="stable")
    cols = [cols[i] for i in order]
    obs = [obs[i] for i in order]
    priors = np.asarray(priors, dtype=np.float64)[order]
    h_ptr = np.zeros(len(cols) + 1, dtype=np.int32)
    h_ptr[1:] = np.cumsum([len(c) for c in cols])
    l_ptr = np.zeros(len(cols) + 1, dtype=np.int32)
    l_ptr[1:] = np.cumsum([len(o) for o in obs])
    h_idx = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    l_idx = (np.concatenate(obs).astype(np.int32) if sum(len(o) for o in obs)
             else np.zeros(0, np.int32))
    n_rows = w * n_rounds
    det_round = (np.arange(n_rows) // w).astype(np.int32)
    return DEM(name, n_rows, len(cols), n_obs, w, n_rounds, h_ptr, h_idx, l_ptr,
               l_idx, priors, det_round, info)


# ------------------------------------------------------------ phenomenological

def phenomenological_dem(code: BBCode, noisy_rounds: int, p: float, q: float,
                         use_hx: bool = True) -> DEM:
    """Data flips (prior p) before each of the noisy rounds and measurement flips
    (prior q) in each noisy round, then one perfect round with no new faults.

    The checks are H_X (Z-type data flips) when use_hx, else H_Z.
    """
    h = code.hx if use_hx else code.hz
    other = code.hz if use_hx else code.hx
    lg = logical_operators(h, other)
    w, n = h.shape
    cols, obs, pri = [], [], []
    for r in range(noisy_rounds):
        for i in range(n):
            cols.append(r * w + np.nonzero(h[:, i])[0])
            obs.append(np.nonzero(lg[:, i])[0])
            pri.append(p)
        for j in range(w):
            cols.append(np.array([r * w + j, (r + 1) * w + j]))
            obs.append(np.zeros(0, dtype=np.int64))
            pri.append(q)
    return _from_columns(f"{code.name} phenomenological p={p} q={q}", cols, obs,
                         pri, w, noisy_rounds + 1, lg.shape[0],
                         dict(model="phenomenological", p=p, q=q,
                              noisy_rounds=noisy_rounds, logicals=lg))


# ------------------------------------------------------------ one-round models

def data_noise_dem(code: BBCode, p_d: float) -> DEM:
    """Appendix A: X-type data-qubit noise only, each data qubit flipped with
    probability p_d (the classical BSC(p_d)), one noiseless syndrome
    measurement: one detector round with H = H_X and the logical operators as
    observables."""
    h = code.hx
    lg = logical_operators(code.hx, code.hz)
    w, n = h.shape
    cols = [np.nonzero(h[:, i])[0] for i in range(n)]
    obs = [np.nonzero(lg[:, i])[0] for i in range(n)]
    return _from_columns(f"{code.name} data noise p_d={p_d}", cols, obs, [p_d] * n, w, 1,
                         lg.shape[0], dict(model="data_noise", p_d=p_d, logicals=lg))


def single_shot_dem(code: BBCode, p_d: float, p_s: float) -> DEM:
    """Appendix B: data flips BSC(p_d) and one noisy syndrome measurement whose
    bits flip with probability p_s. The decoding matrix is [H_X | I]: one
    virtual column per check for its syndrome flip. A correction is right when
    its data part has the same syndrome as the data error and no logical effect
    (Appendix B), so the observables are the logical operators on the data
    columns followed by H_X itself on the data columns (the virtual columns
    touch no observable)."""
    h = code.hx
    lg = logical_operators(code.hx, code.hz)
    w, n = h.shape
    k = lg.shape[0]
    cols, obs, pri = [], [], []
    for i in range(n):
        rows = np.nonzero(h[:, i])[0]
        cols.append(rows)
        obs.append(np.concatenate([np.nonzero(lg[:, i])[0], k + rows]))
        pri.append(p_d)
    for j in range(w):
        cols.append(np.array([j]))
        obs.append(np.zeros(0, dtype=np.int64))
        pri.append(p_s)
    return _from_columns(f"{code.name} single shot p_d={p_d} p_s={p_s}", cols, obs, pri, w, 1,
                         k + w, dict(model="single_shot", p_d=p_d, p_s=p_s, logicals=lg))


# ------------------------------------------------------------ circuit level
#
# Qubit layout: X-check ancillas [0, w), L data [w, 2w), R data [2w, 3w),
# Z-check ancillas [3w, 4w). X-check alpha touches L_{alpha+a_i}, R_{alpha+b_j};
# Z-check gamma touches L_{gamma-b_j}, R_{gamma-a_i} (H_Z = [B^T|A^T]).
#
# One cycle is 8 time steps. Step 0: Z-ancilla reset (and the previous cycle's
# X-ancilla measurement). Steps 1..7: seven CNOT layers; the X ancillas use
# layers 1..6 (their reset shares step 1 with the Z ancillas' first CNOT), the Z
# ancillas layers 0..5 (their measurement shares step 7 with the X ancillas' last
# CNOT). The layer of each of the 12 terms was chosen by exhaustive search so
# that no qubit is used twice in a step and every X-check/Z-check pair overlaps
# on an even number of qubits where the X-check acts first, which makes the
# interleaved X and Z measurements commute (``schedule_is_valid``).

# Term layers: X: (A0, A1, A2, B0, B1, B2); Z: (B0^T, B1^T, B2^T, A0^T, A1^T, A2^T).
DEFAULT_SCHEDULE = ((1, 3, 5, 2, 4, 6), (4, 2, 0, 5, 3, 1))


def _term_maps(code: BBCode):
    l, m = code.l, code.m
    w = l * m

    def shift(idx, da, db):
        a, b = divmod(idx, m)
        return ((a + da) % l) * m + (b + db) % m

    alpha = np.arange(w)
    x_targets = []   # per X term: data qubit for X-check alpha
    for (da, db) in code.a_terms:
        x_targets.append(w + np.array([shift(i, da, db) for i in alpha]))
    for (da, db) in code.b_terms:
        x_targets.append(2 * w + np.array([shift(i, da, db) for i in alpha]))
    z_sources = []   # per Z term: data qubit for Z-check gamma
    for (da, db) in code.b_terms:
        z_sources.append(w + np.array([shift(i, -da, -db) for i in alpha]))
    for (da, db) in code.a_terms:
        z_sources.append(2 * w + np.array([shift(i, -da, -db) for i in alpha]))
    return x_targets, z_sources


def schedule_is_valid(code: BBCode, schedule=DEFAULT_SCHEDULE) -> bool:
    """Checks the circuit: each step uses each qubit at most once, the CNOTs of
    each check reproduce its row of H_X / H_Z, and for every X/Z check pair the
    number of shared data qubits touched first by the X check is even."""
    tx, tz = schedule
    w = code.w
    x_targets, z_sources = _term_maps(code)
    for layer in range(7):
        used = []
        for k in range(6):
            if tx[k] == layer:
                used.append(x_targets[k])
            if tz[k] == layer:
                used.append(z_sources[k])
        if used:
            u = np.concatenate(used)
            if len(np.unique(u)) != len(u):
                return False
    hx = np.zeros((w, 2 * w), np.uint8)
    hz = np.zeros((w, 2 * w), np.uint8)
    for k in range(6):
        hx[np.arange(w), x_targets[k] - w] ^= 1
        hz[np.arange(w), z_sources[k] - w] ^= 1
    if not (np.array_equal(hx, code.hx) and np.array_equal(hz, code.hz)):
        return False
    # time at which X-check alpha / Z-check gamma touch data qubit q
    tx_q = np.full((w, 2 * w), -1)
    tz_q = np.full((w, 2 * w), -1)
    for k in range(6):
        tx_q[np.arange(w), x_targets[k] - w] = tx[k]
        tz_q[np.arange(w), z_sources[k] - w] = tz[k]
    for a in range(w):
        both = (tx_q[a][None, :] >= 0) & (tz_q >= 0)
        first = both & (tx_q[a][None, :] < tz_q)
        if np.any(first.sum(axis=1) % 2):
            return False
    return True


def _circuit_faults(code: BBCode, rounds: int, p: float, schedule):
    """Yields the moment list and the fault list (moment, stage, qubits, prob).

    stage 0: injected after the moment's resets and gates; stage 1: injected
    before the moment's measurements (measurement flips).
    """
    w = code.w
    tx, tz = schedule
    x_targets, z_sources = _term_maps(code)
    xa = np.arange(w)
    za = 3 * w + np.arange(w)
    data = np.arange(w, 3 * w)
    moments = []
    faults = []
    p1 = 2.0 * p / 3.0     # X part of single-qubit depolarising
    p2 = 4.0 * p / 15.0    # each X part of two-qubit depolarising
    for r in range(rounds):
        for step in range(8):
            mo = dict(reset_z=[], reset_x=[], cnots=[], meas_z=[], round=r, step=step)
            busy = set()
            if step == 0:
                mo["reset_z"] = za
                busy.update(za.tolist())
                t = len(moments)
                for q in za:
                    faults.append((t, 0, (int(q),), p))           # reset flip
                if r == 0:
                    mo["reset_d"] = data                           # data |0>
                    for q in data:
                        faults.append((t, 0, (int(q),), p))
                else:
                    for q in data:
                        faults.append((t, 0, (int(q),), p1))      # idle
            else:
                layer = step - 1
                t = len(moments)
                if layer == 0:
                    mo["reset_x"] = xa                            # |+>: no X part
                    busy.update(xa.tolist())
                if layer == 6:
                    mo["meas_z"] = za
                    busy.update(za.tolist())
                    for q in za:
                        faults.append((t, 1, (int(q),), p))       # meas flip
                cn = []
                for k in range(6):
                    if tx[k] == layer:
                        cn += list(zip(xa.tolist(), x_targets[k].tolist()))
                    if tz[k] == layer:
                        cn += list(zip(z_sources[k].tolist(), za.tolist()))
                mo["cnots"] = cn
                for (c, tq) in cn:
                    busy.add(c)
                    busy.add(tq)
                    faults.append((t, 0, (c,), p2))
                    faults.append((t, 0, (tq,), p2))
                    faults.append((t, 0, (c, tq), p2))
                for q in range(4 * w):
                    if q not in busy:
                        faults.append((t, 0, (q,), p1))
            moments.append(mo)
    return moments, faults


def circuit_dem(code: BBCode, rounds: int, p: float, schedule=DEFAULT_SCHEDULE,
                merge: bool = True) -> DEM:
    """Circuit-level DEM for Z-check detectors (X-type faults), Z-basis memory.

    Detector round r < rounds: Z-check outcome of cycle r XOR cycle r-1 (cycle 0
    alone); detector round `rounds`: the noiseless final syndrome H_Z x computed
    from the data measurement, XOR the last cycle's outcome. Observables:
    L_Z x with L_Z a basis of ker(H_X) modulo rowspace(H_Z).
    """
    if not schedule_is_valid(code, schedule):
        raise ValueError("invalid syndrome-extraction schedule")
    w = code.w
    nq = 4 * w
    moments, faults = _circuit_faults(code, rounds, p, schedule)
    nf = len(faults)
    nwords = (nf + 63) // 64
    frames = np.zeros((nq, nwords), dtype=np.uint64)
    by_moment = {}
    for f, (t, stage, qs, pr) in enumerate(faults):
        by_moment.setdefault((t, stage), []).append((f, qs))
    meas = []
    one = np.uint64(1)
    for t, mo in enumerate(moments):
        for key in ("reset_z", "reset_x", "reset_d"):
            if key in mo and len(mo[key]):
                frames[np.asarray(mo[key])] = 0
        if mo["cnots"]:
            cn = np.array(mo["cnots"])
            frames[cn[:, 1]] ^= frames[cn[:, 0]]
        for (f, qs) in by_moment.get((t, 0), []):
            for q in qs:
                frames[q, f >> 6] ^= one << np.uint64(f & 63)
        for (f, qs) in by_moment.get((t, 1), []):
            for q in qs:
                frames[q, f >> 6] ^= one << np.uint64(f & 63)
        if len(mo["meas_z"]):
            meas.append(frames[np.asarray(mo["meas_z"])].copy())
    assert len(meas) == rounds
    data_frame = frames[w:3 * w]
    dets = [meas[0]]
    for r in range(1, rounds):
        dets.append(meas[r] ^ meas[r - 1])
    # final noiseless syndrome from data, XOR last cycle outcome
    hz = code.hz
    final = np.zeros((w, nwords), dtype=np.uint64)
    for g in range(w):
        for q in np.nonzero(hz[g])[0]:
            final[g] ^= data_frame[q]
    dets.append(final ^ meas[rounds - 1])
    det_bits = np.concatenate(dets, axis=0)                     # [n_rows, nwords]
    lz = logical_operators(code.hz, code.hx)
    obs_bits = np.zeros((lz.shape[0], nwords), dtype=np.uint64)
    for k in range(lz.shape[0]):
        for q in np.nonzero(lz[k])[0]:
            obs_bits[k] ^= data_frame[q]

    def unpack(bits):
        b = bits.view(np.uint8).reshape(bits.shape[0], -1)
        u = np.unpackbits(b, axis=1, bitorder="little")
        return u[:, :nf].astype(bool)

    det_mat = unpack(det_bits)      # [n_rows, nf]
    obs_mat = unpack(obs_bits)      # [K, nf]
    priors = np.array([f[3] for f in faults])
    cols, obs, pri = [], [], []
    index = {}
    dropped_mass = 0.0
    dropped_logical = 0.0
    for f in range(nf):
        rows = np.nonzero(det_mat[:, f])[0]
        ob = np.nonzero(obs_mat[:, f])[0]
        if rows.size == 0:
            dropped_mass += priors[f]
            if ob.size:
                dropped_logical += priors[f]
            continue
        key = (rows.tobytes(), ob.tobytes())
        if merge and key in index:
            c = index[key]
            p0 = pri[c]
            pri[c] = p0 + priors[f] - 2.0 * p0 * priors[f]
        else:
            index[key] = len(cols)
            cols.append(rows)
            obs.append(ob)
            pri.append(priors[f])
    span = [int((c[-1] // w) - (c[0] // w)) for c in cols]
    info = dict(model="circuit", p=p, noisy_rounds=rounds, raw_faults=nf,
                dropped_mass=dropped_mass, dropped_logical_mass=dropped_logical,
                max_span=max(span) if span else 0, schedule=schedule, logicals=lz)
    return _from_columns(f"{code.name} circuit p={p} R={rounds}", cols, obs, pri, w,
                         rounds + 1, lz.shape[0], info)


def round_shapes(dem: DEM) -> dict:
    """Counts of columns by (first round, span): the H'_0/H_0/H_1 block widths."""
    fr = dem.first_round()
    lr = dem.last_round()
    out = {}
    for f, l in zip(fr.tolist(), lr.tolist()):
        out[(f, l - f)] = out.get((f, l - f), 0) + 1
    return out
