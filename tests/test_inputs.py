"""Input generators: BB codes, GF(2) algebra, DEMs and the Philox sampler.

These pin the shared input side (codes, noise models, shots) against facts the
paper and the mathematics fix.
"""
import os

import numpy as np
import pytest

from gdg_inputs.bb import CODE_K, CODES, get_code, gf2_rank, gf2_nullspace, logical_operators
from gdg_inputs.dem import (DEFAULT_SCHEDULE, circuit_dem, phenomenological_dem, round_shapes,
                            schedule_is_valid)
from gdg_inputs.philox import philox4x32_10, sample_errors, syndromes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("key", list(CODES))
def test_bb_css_and_k(key):
    c = get_code(key)
    assert not ((c.hx.astype(int) @ c.hz.T.astype(int)) % 2).any()      # H_X H_Z^T = 0
    assert c.k() == CODE_K[key]                                          # k from GF(2) ranks
    assert (c.hx.sum(0) == 3).all() and (c.hx.sum(1) == 6).all()         # weights 3 / 6
    assert (c.hz.sum(0) == 3).all() and (c.hz.sum(1) == 6).all()


def test_bb288_first_columns():
    # Appendix B: the first columns of A and B for N=288 are y^5+y^10+x^9 and
    # y^9+x^10+x^11, with x^a y^b at position 12a+b.
    c = get_code("288")
    assert sorted(np.nonzero(c.a[:, 0])[0].tolist()) == sorted([5, 10, 12 * 9])
    assert sorted(np.nonzero(c.b[:, 0])[0].tolist()) == sorted([9, 12 * 10, 12 * 11])


def test_bb288_syndrome_code_counts():
    # Appendix B: 288 columns of weight 3; each column is b_i x^a y^b.
    c = get_code("288")
    cols = {tuple(np.nonzero(c.hx[:, j])[0]) for j in range(288)}
    assert len(cols) == 288


def test_gf2_helpers():
    rng = np.random.default_rng(1)
    for _ in range(20):
        a = rng.integers(0, 2, (7, 11)).astype(np.uint8)
        ns = gf2_nullspace(a)
        assert ns.shape[0] == 11 - gf2_rank(a)
        assert not ((a.astype(int) @ ns.T.astype(int)) % 2).any()


@pytest.mark.parametrize("key", ["72", "144"])
def test_logicals(key):
    c = get_code(key)
    lz = logical_operators(c.hz, c.hx)        # Z-type logicals: ker(H_X) mod rowspace(H_Z)
    assert lz.shape[0] == CODE_K[key]
    assert not ((c.hx.astype(int) @ lz.T.astype(int)) % 2).any()
    assert gf2_rank(np.vstack([c.hz, lz])) == gf2_rank(c.hz) + CODE_K[key]


def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        lines = [l for l in f if l.strip() and not l.startswith("#")]
    assert len(lines) == 3
    for line in lines:
        v = [int(x, 16) for x in line.split()]
        out = philox4x32_10(*[np.uint32(x) for x in v[:6]])
        assert [int(o) for o in out] == v[6:]


def test_sampler_rates_and_determinism():
    thr = np.array([int(p * 2 ** 32) for p in (0.5, 0.1, 0.01, 0.0, 0.25)], np.uint32)
    e = sample_errors(thr, 20000, seed=7)
    rates = e.mean(0)
    for r, p in zip(rates, (0.5, 0.1, 0.01, 0.0, 0.25)):
        assert abs(r - p) <= 5 * np.sqrt(p * (1 - p) / 20000) + 1e-12
    assert np.array_equal(e, sample_errors(thr, 20000, seed=7))
    # shots are addressed by index: a later chunk equals the tail of a longer draw
    assert np.array_equal(e[500:700], sample_errors(thr, 200, seed=7, shot0=500))
    assert not np.array_equal(e, sample_errors(thr, 20000, seed=8))


def test_phenomenological_structure():
    c = get_code("72")
    d = phenomenological_dem(c, 6, 0.005, 0.005)
    assert d.n_rows == 7 * 36 and d.n_cols == 6 * (72 + 36)
    deg = np.diff(d.h_ptr)
    assert sorted(set(deg.tolist())) == [2, 3]          # measurement faults: degree 2 (Sec. II-B)
    span = d.last_round() - d.first_round()
    assert span.max() <= 1
    e = sample_errors(d.thresholds(), 50, seed=3)
    det, obs = syndromes(d, e)
    h = d.dense_h().astype(int)
    assert np.array_equal(det, (e.astype(int) @ h.T) % 2)


@pytest.mark.parametrize("key", list(CODES))
def test_schedule_valid(key):
    assert schedule_is_valid(get_code(key), DEFAULT_SCHEDULE)


def test_schedule_rejects_bad():
    # swapping two Z layers breaks the X/Z interleaving condition or a qubit clash
    tx, tz = DEFAULT_SCHEDULE
    bad = (tx, (tz[1], tz[0]) + tz[2:])
    assert not schedule_is_valid(get_code("72"), bad)


@pytest.mark.parametrize("key", ["72", "144"])
def test_circuit_dem_structure(key):
    c = get_code(key)
    w = c.w
    d = circuit_dem(c, 6, 0.002)
    span = d.last_round() - d.first_round()
    assert span.max() <= 1                        # no fault spans more than two rounds (Sec. II-B)
    assert d.info["dropped_logical_mass"] == 0.0  # no undetectable logical fault at first order
    sh = round_shapes(d)
    assert sh[(0, 0)] == 2 * w                    # H'_0 is w x 2w (Appendix D)
    for r in range(1, 6):
        assert sh[(r, 0)] == 3 * w                # H_0 is w x 3w (Fig. 1 caption)
    # measurement flips of the Z ancillas are degree-2 columns on one check
    deg = np.diff(d.h_ptr)
    assert (deg == 2).sum() > 0
    # sampled detectors are H e
    e = sample_errors(d.thresholds(), 20, seed=3)
    det, obs = syndromes(d, e)
    assert np.array_equal(det, (e.astype(int) @ d.dense_h().astype(int).T) % 2)
    assert np.array_equal(obs, (e.astype(int) @ d.dense_l().astype(int).T) % 2)
