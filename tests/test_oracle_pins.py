"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test would fail for a plausible mistake in the oracle: a dropped term or
wrong sign in Eqs. 1-3 (hand example, tree exactness), a wrong history rule or
tie-break in Alg. 1, wrong thresholds in Alg. 3, a wrong bit order in Alg. 2
(Fig. 2 labels), order dependence in peeling, a wrong window slice, commit or
path metric (brute force, Eq. 7/8 composition).
"""
import itertools
import os

import numpy as np
import pytest

from gdg_inputs.bb import get_code, logical_operators
from gdg_inputs.dem import circuit_dem, phenomenological_dem
from gdg_inputs.philox import sample_errors, syndromes
from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_cases(name):
    cases, cur = [], None
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, _, v = line.partition(" ")
        if k == "case":
            cur = {}
            cases.append(cur)
        elif k == "H":
            cur[k] = np.array([[int(x) for x in r.split(",")] for r in v.split(";")], np.uint8)
        else:
            cur[k] = np.array([float(x) for x in v.split()])
    return cases


def test_eq1_4_hand_example():
    A, B = _read_cases("minsum_3vn_2cn.txt")
    prm = O.params(alpha=0.625)
    post = O.dense_bp(A["H"], A["llr"], A["syn"].astype(np.uint8), prm, 2)
    np.testing.assert_allclose(post[0], A["post1"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(post[1], A["post2"], rtol=0, atol=1e-15)
    post = O.dense_bp(B["H"], B["llr"], B["syn"].astype(np.uint8), prm, 1)
    np.testing.assert_allclose(post[0], B["post1"], rtol=0, atol=1e-15)
    pm, e, fl = O.dense_gdg(B["H"], B["llr"], B["syn"].astype(np.uint8), prm)
    assert e.tolist() == B["ehat"].astype(int).tolist()
    assert pm == B["pm"][0] and fl & 1


def _random_tree(rng, n_vn, max_cn_deg=4):
    """Tanner tree: connected, acyclic, every CN of degree >= 2."""
    H_rows = []
    vn = 1
    frontier = [0]
    while vn < n_vn:
        anchor = int(rng.choice(frontier))
        k = int(rng.integers(1, max_cn_deg))
        k = min(k, n_vn - vn)
        row = [anchor] + list(range(vn, vn + k))
        frontier += list(range(vn, vn + k))
        vn += k
        H_rows.append(row)
    H = np.zeros((len(H_rows), n_vn), np.uint8)
    for r, cols in enumerate(H_rows):
        H[r, cols] = 1
    return H


def _brute(H, llr, syn):
    m, n = H.shape
    best0 = np.full(n, np.inf)
    best1 = np.full(n, np.inf)
    z0 = np.zeros(n)
    z1 = np.zeros(n)
    p = 1.0 / (1.0 + np.exp(llr))                   # prior flip probability
    for bits in itertools.product([0, 1], repeat=n):
        e = np.array(bits)
        if (((H.astype(int) @ e) % 2) != syn).any():
            continue
        cost = float(llr @ e)
        w = float(np.prod(np.where(e == 1, p, 1 - p)))
        best1 = np.where(e == 1, np.minimum(best1, cost), best1)
        best0 = np.where(e == 0, np.minimum(best0, cost), best0)
        z1 += np.where(e == 1, w, 0.0)
        z0 += np.where(e == 0, w, 0.0)
    return best1 - best0, np.log(z0 / z1)


@pytest.mark.parametrize("seed", range(12))
def test_tree_minsum_is_min_marginal_and_sumproduct_is_exact(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 12))
    H = _random_tree(rng, n)
    llr = rng.uniform(0.3, 3.0, n)
    e = (rng.random(n) < 0.3).astype(int)
    syn = ((H.astype(int) @ e) % 2).astype(np.uint8)
    minm, marg = _brute(H, llr, syn)
    iters = 2 * n + 2                               # more than the tree diameter
    post_ms = O.dense_bp(H, llr, syn, O.params(alpha=1.0), iters)[-1]
    post_sp = O.dense_bp(H, llr, syn, O.params(alpha=1.0, sum_product=1), iters)[-1]
    np.testing.assert_allclose(post_ms, minm, rtol=0, atol=1e-9)
    np.testing.assert_allclose(post_sp, marg, rtol=0, atol=1e-9)


def _ranking_order_ok(kept, key, n_keep, tol=1e-9):
    """kept lists the n_keep columns of smallest key in ascending key order,
    equal keys (within tol) in ascending column order."""
    if len(kept) != n_keep:
        return False
    for a, b in zip(kept[:-1], kept[1:]):
        if key[a] > key[b] + tol or (abs(key[a] - key[b]) <= tol and a > b):
            return False
    last = kept[-1]
    for c in set(range(len(key))) - set(kept.tolist()):
        if key[c] < key[last] - tol or (abs(key[c] - key[last]) <= tol and c < last):
            return False
    return True


def _tie_tree():
    """A tree with symmetric leaves of equal prior: columns 1 and 2 (on CN 0)
    and 6 and 7 (on CN 2) have identical min-marginals by symmetry."""
    H = np.zeros((3, 8), np.uint8)
    H[0, [0, 1, 2, 3]] = 1
    H[1, [3, 4, 5]] = 1
    H[2, [5, 6, 7]] = 1
    llr = np.array([2.1, 0.7, 0.7, 1.3, 2.6, 0.9, 1.6, 1.6])
    syn = np.array([1, 0, 1], np.uint8)
    return H, llr, syn


@pytest.mark.parametrize("pre_iters", [8, 16])
@pytest.mark.parametrize("seed", list(range(10)) + ["ties"])
def test_preprocessing_ranking_on_trees(seed, pre_iters):
    """Preprocessing, ranking and truncation (Sec. III, last paragraphs; Sec.
    IV-C) through decode_window itself. On a tree Tanner graph (alpha = 1, no
    clipping reached) flooding min-sum reaches the exact min-marginal
    differences within five iterations and stays there, so the ranking key of
    every column -- the sum of its last four preprocessing posteriors -- must be
    4 x the brute-force min-marginal. An extra check row with no columns and
    syndrome 1 keeps the preprocessing from stopping early. The kept columns are
    then the trunc_factor * m smallest keys in ascending order, equal keys by
    ascending column index. A descending sort, a sum over all pre_iters
    iterations or over other than the last four, or another tie rule fails."""
    if seed == "ties":
        H, llr, syn = _tie_tree()
    else:
        rng = np.random.default_rng(100 + seed)
        n = int(rng.integers(6, 12))
        H = _random_tree(rng, n)
        llr = rng.uniform(0.3, 3.0, n)
        e = (rng.random(n) < 0.3).astype(int)
        syn = ((H.astype(int) @ e) % 2).astype(np.uint8)
    n = H.shape[1]
    minm, _ = _brute(H, llr, syn)
    post = O.dense_bp(H, llr, syn, O.params(alpha=1.0), pre_iters)
    assert np.abs(post[4:] - minm).max() < 1e-12        # converged from iteration 5 on
    assert np.abs(post[0] - minm).max() > 1e-6          # but not after the first
    Hd = np.vstack([H, np.zeros((1, n), np.uint8)])
    sd = np.append(syn, 1).astype(np.uint8)
    m = Hd.shape[0]
    for tf in (1, 2):
        if tf * m >= n:
            continue
        r = O.dense_window(Hd, llr, sd, O.params(alpha=1.0, pre_iters=pre_iters, trunc_factor=tf))
        np.testing.assert_allclose(r["lsum"], 4 * minm, rtol=0, atol=1e-9)
        assert _ranking_order_ok(r["kept"], 4 * minm, tf * m), (r["kept"], 4 * minm)
        # the same order with the oracle's own keys, exact ties included
        assert _ranking_order_ok(r["kept"], r["lsum"], tf * m, tol=0.0)
    if seed == "ties":
        # keys -0.4 for columns 3 and 5, +0.4 for 1, 2, 6 and 7 (exactly equal):
        # the four kept columns are 3, 5, then the two lowest of the tied four
        assert r["lsum"][1] == r["lsum"][2] == r["lsum"][6] == r["lsum"][7]
        assert r["lsum"][3] == r["lsum"][5]
        assert r["kept"].tolist() == [3, 5, 1, 2]


def test_alg3_unsatisfied_cn_wiring():
    """Alg. 3's unsatisfied-CN count inside run_path (reading R10: an active CN
    whose residual syndrome differs from the XOR of its active neighbours'
    current hard decisions, from the state after the step's BP and before the
    pass). On random frustrated graphs the count the oracle uses equals one
    recomputed here from H, the syndrome, the statuses and the Eq. 4 hard
    decisions of the step's posteriors; and every eligible VN whose four history
    posteriors lie in (3, 30] is decided 0 exactly when at least 3 of its CNs
    are unsatisfied (P_D = 3). Both outcomes must occur, including the
    boundary counts 3 (decided) and 2 (not decided)."""
    seen = {}
    for seed in range(40):
        rng = np.random.default_rng(seed)
        m, n = 24, 48
        H = np.zeros((m, n), np.uint8)
        for c in range(n):
            H[rng.choice(m, int(rng.integers(3, 5)), replace=False), c] = 1
        llr = rng.uniform(1.0, 6.0, n)
        e = (rng.random(n) < 0.12).astype(int)
        syn = ((H.astype(int) @ e) % 2).astype(np.uint8)
        r = O.dense_path_probe(H, llr, syn, O.params(alpha=1.0, g=0, low_error=0, dmax_main=6))
        Hi = H.astype(np.int64)
        for i in range(r["steps"]):
            st = r["status"][i]
            act = st < 0
            e_now = np.where(act, (r["post"][i] <= 0).astype(int), np.maximum(st, 0))
            unsat = (Hi @ e_now + syn) % 2
            nu = Hi.T @ unsat
            assert np.array_equal(nu[act], r["n_unsat"][i][act]), (seed, i)
            for c in np.nonzero(act & (H.sum(0) >= 3))[0]:
                if 3.0 < r["hmin"][i][c] <= 30.0:
                    want = 0 if nu[c] >= 3 else -1
                    assert r["agg"][i][c] == want, (seed, i, c, nu[c], r["agg"][i][c])
                    seen[int(min(nu[c], 3))] = seen.get(int(min(nu[c], 3)), 0) + 1
    assert seen.get(3, 0) > 0 and seen.get(2, 0) > 0, seen


def test_alg1_select_vn_table():
    # columns: hist (4 posteriors), degree, status
    h = np.array([[-1, -1, -1, -1],     # 0: all <= 0, sum -4
                  [5, -10, -10, 5],     # 1: sum -10 but not all <= 0
                  [-2, -2, -2, -2],     # 2: all <= 0, sum -8, but degree 2
                  [-3, -3, -3, -3],     # 3: all <= 0, sum -12, but decimated
                  [-1, -1, -1, -1.0]], np.float64)   # 4: ties with 0 -> 0 wins (lower index)
    deg = [3, 3, 2, 3, 4]
    st = [-1, -1, -1, 1, -1]
    g, f, _ = O.select_vn(h, deg, st, [0] * 5, True, 1, True)
    assert (g, f) == (0, 1)
    # no all-nonpositive candidate: the smallest sum, favoured value from its sign
    h2 = np.array([[1, 1, 1, 1], [2, -1, 0.5, 0.1], [1, -3, 1, -3]], np.float64)
    g, f, _ = O.select_vn(h2, [3, 3, 3], [-1] * 3, [0] * 3, True, 1, True)
    assert (g, f) == (2, 1)             # sum -4 <= 0 -> value 1
    g, f, _ = O.select_vn(h2[:2], [3, 3], [-1] * 2, [0] * 2, True, 1, True)
    assert (g, f) == (1, 0)             # sum 1.6 > 0 -> value 0
    # nothing eligible
    g, f, _ = O.select_vn(h2, [2, 1, 2], [-1] * 3, [0] * 3, True, 1, True)
    assert g == -1
    # exact-zero sum: favoured value 1 (Eq. 4 convention)
    g, f, _ = O.select_vn(np.array([[1, -1, 2, -2.0]]), [3], [-1], [0], True, 1, True)
    assert (g, f) == (0, 1)


def test_alg3_thresholds():
    # Alg. 3: P_A=-3 / 0, P_B=-12 / -10 (-16 at D=1), P_C=30, P_D=3.
    A = O.agg_dec
    assert A([-4, -4, -4, -4], 2, True, 0) == 1          # all < -3, sum -16 < -12
    assert A([-4, -4, -4, -0.5], 2, True, 0) == -1       # one value >= -3
    assert A([-3.5, -3.5, -3.5, -3.5], 2, True, 0) == 1  # sum -14 < -12
    assert A([-3.5, -3.5, -3.5, -3.5], 1, True, 0) == -1  # D=1: P_B=-16
    assert A([-2.6, -2.6, -2.6, -2.6], 2, False, 0) == 1   # off main: P_A=0, P_B=-10
    assert A([-2.4, -2.4, -2.4, -2.4], 2, False, 0) == -1  # sum -9.6 >= -10
    assert A([31, 31, 31, 31], 4, True, 0) == 0          # > P_C at D <= 4
    assert A([31, 31, 31, 31], 5, True, 0) == -1         # D > 4 and too few unsatisfied CNs
    assert A([3.5, 4, 5, 6], 5, True, 3) == 0            # > P_D with >= 3 unsatisfied CNs
    assert A([3.5, 4, 5, 6], 5, True, 2) == -1
    assert A([2.5, 4, 5, 6], 5, True, 3) == -1
    # Alg. 3 inside Alg. 1: decided VNs leave the selection
    h = np.array([[-5, -5, -5, -5], [-1, -1, -1, -1.0]])
    g, f, agg = O.select_vn(h, [3, 3], [-1, -1], [0, 0], False, 2, True)
    assert agg.tolist() == [1, -1] and (g, f) == (1, 1)


def test_alg2_path_rule_fig2_labels():
    prm = O.params(g=4, dmax_main=25, extra_steps=10)
    assert O.n_paths(prm) == 16
    # Under the figure's all-favoured-is-one demonstration (f = 1): the main path
    # (id 0) takes 1 at every depth, id 1 is the side path splitting at depth 4,
    # the leftmost leaf id 15 takes the unfavoured value at all four depths, and
    # ids 8..15 form the left subtree of the root.
    def seq(pid):
        return [O.path_value(prm, pid, D, 1)[0] for D in range(1, 8)]
    assert seq(0) == [1] * 7
    assert seq(1) == [1, 1, 1, 0, 1, 1, 1]
    assert seq(15) == [0, 0, 0, 0, 1, 1, 1]
    assert seq(2) == [1, 1, 0, 1, 1, 1, 1]
    for pid in range(8, 16):
        assert seq(pid)[0] == 0
    for pid in range(0, 8):
        assert seq(pid)[0] == 1
    # favoured value 0 flips the taken values
    assert [O.path_value(prm, 5, D, 0)[0] for D in range(1, 5)] == [0, 1, 0, 1]
    # D_max: 25 on main, 4 + 10 on every tree / side path
    assert O.path_value(prm, 0, 1, 1)[2] == 25
    assert all(O.path_value(prm, p, 1, 1)[2] == 14 for p in range(1, 16))
    # on-main flag (Alg. 3 thresholds) until the first unfavoured decision
    assert O.path_value(prm, 1, 4, 1)[1] is True
    assert O.path_value(prm, 1, 5, 1)[1] is False
    assert O.path_value(prm, 8, 1, 1)[1] is True
    assert O.path_value(prm, 8, 2, 1)[1] is False
    # paper-faithful extra side paths (split at depths 5..10, D_max = split + 10)
    prm2 = O.params(g=4, side_max_depth=10)
    assert O.n_paths(prm2) == 22
    v, om, dm = O.path_value(prm2, 16, 5, 1)
    assert (v, dm) == (0, 15)
    assert O.path_value(prm2, 21, 10, 1)[0] == 0 and O.path_value(prm2, 21, 10, 1)[2] == 20


def test_peel_order_independent_and_contradiction():
    rng = np.random.default_rng(5)
    for trial in range(40):
        m, n = 10, 14
        H = (rng.random((m, n)) < 0.2).astype(np.uint8)
        e = (rng.random(n) < 0.3).astype(int)
        s = ((H.astype(int) @ e) % 2).astype(np.int32)
        status = np.full(n, -1, np.int32)
        dec = rng.choice(n, 6, replace=False)
        status[dec] = e[dec]                      # consistent decimations
        s_res = (s + H[:, dec].astype(int) @ e[dec]) % 2
        ok, st, ss = O.peel(H, status, s_res)
        assert ok                                  # consistent data never contradicts
        decided = st >= 0
        assert (st[decided] == e[decided]).all()   # peeling recovers e (consistent data)
        # every degree-one CN is resolved
        act = st < 0
        assert not ((H[:, act].sum(1) == 1)).any()
        # relabelling rows and columns gives the same closure
        pr, pc = rng.permutation(m), rng.permutation(n)
        ok2, st2, ss2 = O.peel(H[pr][:, pc], status[pc], s_res[pr])
        assert ok2 and np.array_equal(st2, st[pc]) and np.array_equal(ss2, ss[pr])
    # contradiction: two degree-one checks on one VN with different syndromes
    H = np.array([[1, 0], [1, 0], [0, 1]], np.uint8)
    ok, _, _ = O.peel(H, np.array([-1, -1]), np.array([1, 0, 0]))
    assert not ok
    # a check left with no active neighbour and residual 1
    ok, _, _ = O.peel(np.array([[1, 1]], np.uint8), np.array([0, 0]), np.array([1]))
    assert not ok


def test_bruteforce_code_capacity_72():
    """Every weight <= 2 fault on H_X of [[72,12,6]] (72 + 2556 patterns) is decoded to
    the minimum path metric and to a logically equivalent correction."""
    c = get_code("72")
    H = c.hx
    n = 72
    llr = np.full(n, np.log(0.99 / 0.01))
    L = logical_operators(c.hx, c.hz)
    pats = [(i,) for i in range(n)] + list(itertools.combinations(range(n), 2))
    for g in (0, 4):
        prm = O.params(alpha=0.625, g=g)
        for pat in pats:
            e = np.zeros(n, np.uint8)
            e[list(pat)] = 1
            s = ((H.astype(int) @ e) % 2).astype(np.uint8)
            pm, eh, fl = O.dense_gdg(H, llr, s, prm)
            r = (eh ^ e).astype(int)
            assert abs(pm - len(pat) * llr[0]) < 1e-9, pat
            assert not ((H.astype(int) @ r) % 2).any() and not ((L.astype(int) @ r) % 2).any()


@pytest.mark.parametrize("k", [1, 4])
def test_bruteforce_c1_window(k):
    """All weight <= 2 fault patterns of a [[72,12,6]] phenomenological window
    (middle window: 324 columns, 52650 patterns; last window: 216 columns).
    The decoded PM equals the brute-force minimum over all patterns with that
    syndrome, except where every minimum-PM explanation uses only columns of
    degree <= 2: those columns are never eligible in Alg. 1, so GDG can reach them
    only through BP convergence (a limitation of the method, reported here)."""
    dem = phenomenological_dem(get_code("72"), 6, 0.005, 0.005)
    w = O.OracleWindow(dem, k, 3)
    ex = w.export()
    H = ex["H"].astype(np.int64)
    llr = ex["llr"]
    n = w.n
    deg = H.sum(0)
    pats = [(i,) for i in range(n)] + list(itertools.combinations(range(n), 2))
    E = np.zeros((len(pats), n), np.uint8)
    for i, p in enumerate(pats):
        E[i, list(p)] = 1
    S = ((E.astype(np.int64) @ H.T) % 2).astype(np.uint8)
    pm_pat = E @ llr
    keys = [s.tobytes() for s in S]
    best, only_low = {}, {}
    for i, kk in enumerate(keys):
        b = best.get(kk, np.inf)
        low = bool((deg[list(pats[i])] <= 2).all())
        if pm_pat[i] < b - 1e-9:
            best[kk] = pm_pat[i]
            only_low[kk] = low
        elif abs(pm_pat[i] - b) <= 1e-9:
            only_low[kk] = only_low[kk] and low
    bmin = np.array([best[kk] for kk in keys])
    r = w.decode(O.params(alpha=0.625, g=0), S)
    hit = np.abs(r["pm"] - bmin) <= 1e-9
    miss = np.nonzero(~hit)[0]
    for i in miss:
        assert only_low[keys[i]], (pats[i], r["pm"][i], bmin[i])
    assert hit.mean() > 0.995
    # a satisfied decision reproduces its syndrome exactly
    sat = (r["flags"] & 1) == 1
    assert np.array_equal((r["e"][sat].astype(np.int64) @ H.T) % 2, S[sat])


@pytest.mark.parametrize("model", ["phen", "circuit"])
def test_commit_composes_to_eq8(model):
    """Decoding whole shots window by window: the residual detectors the oracle
    reports equal H_circ e_committed + det recomputed here in integer
    arithmetic, the observable check equals L e + l (Eq. 9), and a shot counts as
    a success iff both vanish (Eq. 8 and Eq. 9). Every window flagged satisfied
    leaves its first round's residual detectors at zero (Eq. 7)."""
    if model == "phen":
        dem = phenomenological_dem(get_code("72"), 6, 0.02, 0.02)
        prm = O.params(alpha=0.625)
    else:
        dem = circuit_dem(get_code("72"), 6, 0.004)
        prm = O.params(alpha=1.0, g=4, pre_iters=8, trunc_factor=2, low_error=0)
    e = sample_errors(dem.thresholds(), 200, seed=11)
    det, obs = syndromes(dem, e)
    r = O.decode_shots(dem, 3, prm, det, obs)
    H = dem.dense_h().astype(np.int64)
    L = dem.dense_l().astype(np.int64)
    resid = (det.astype(np.int64) + r["e"].astype(np.int64) @ H.T) % 2
    assert np.array_equal(resid, r["det_out"])
    lres = (obs.astype(np.int64) + r["e"].astype(np.int64) @ L.T) % 2
    assert np.array_equal(lres, r["obs_out"])
    fail = resid.any(1) | lres.any(1)
    assert np.array_equal(fail, r["fail"].astype(bool))
    assert r["fail"].sum() < 200          # the decoder does decode
    w = dem.w
    nwin = dem.n_rounds - 2
    for k in range(nwin - 1):
        sat = (r["win_flags"][:, k] & 1) == 1
        # rows of round k are final after window k; only satisfied windows must clear them
        # (later windows never touch round k again)
        assert not resid[sat][:, k * w:(k + 1) * w].any()


def test_window_shapes_c1():
    dem = phenomenological_dem(get_code("72"), 6, 0.005, 0.005)
    for k in range(5):
        w = O.OracleWindow(dem, k, 3)
        ex = w.export()
        rw = sorted(set(ex["H"].sum(1).tolist()))
        if k < 4:
            assert (w.m, w.n, w.n_edges) == (108, 324, 828) and rw == [7, 8]
            assert ex["commit"].sum() == 108
        else:
            assert (w.m, w.n, w.n_edges) == (108, 216, 576) and rw == [1, 7, 8]
            assert ex["commit"].sum() == 216
    # the merged unit columns of a middle window carry the measurement prior q
    w = O.OracleWindow(dem, 1, 3).export()
    unit = w["src"] < 0
    assert unit.sum() == 36
    np.testing.assert_allclose(w["prior"][unit], 0.005, rtol=1e-12)


def test_unit_column_prior_merge():
    """H_1 -> identity merge: a unit column's prior is the odd-parity
    probability of the spilling columns on its row."""
    dem = circuit_dem(get_code("72"), 4, 0.003)
    w = O.OracleWindow(dem, 0, 3)
    ex = w.export()
    fr, lr = dem.first_round(), dem.last_round()
    spill = np.nonzero((fr == 2) & (lr == 3))[0]
    for u in np.nonzero(ex["src"] < 0)[0]:
        row = -1 - ex["src"][u]                     # local row, in round 2
        cols = [c for c in spill if (row + w.row0) in dem.col_rows(c).tolist()]
        pe = 0.0
        for c in cols:                               # odd number of independent flips
            pe = pe * (1 - dem.priors[c]) + (1 - pe) * dem.priors[c]
        assert abs(ex["prior"][u] - pe) < 1e-15


def test_decided_ones_bound_the_path_metric():
    """The premise of the decoder's branch and bound over paths: a VN a path
    decimates to 1 is 1 in that path's answer (decimation fixes it; Alg. 1 with
    Fig. 2's guesses), so with positive priors the path's Eq. 5 metric is at
    least the sum of the priors of its decisions to 1. Checked on every
    converged path of the oracle's 16-path tree, replayed from its logs."""
    dem = circuit_dem(get_code("72"), 6, 0.004)
    prm = O.params(alpha=1.0, g=4, pre_iters=8, trunc_factor=2, low_error=1, dmax_main=25,
                   extra_steps=10)
    e = sample_errors(dem.thresholds(), 80, seed=5)
    det, _ = syndromes(dem, e)
    w = O.OracleWindow(dem, 0, 3)
    llr = w.export()["llr"]
    assert (llr > 0).all()
    syn = np.ascontiguousarray(det[:, w.row0:w.row0 + w.m])
    out = w.decode(prm, syn, logs=True)
    checked = 0
    for s in range(syn.shape[0]):
        if out["ends"][s, :, 1].max() == 0:
            continue   # met the syndrome in the preprocessing: no paths
        for p in range(out["dec"].shape[1]):
            d = out["dec"][s, p]
            steps = int((d[:, 0] >= 0).sum())
            r = w.replay(prm, syn[s], out["sel"][s], p, d[:steps, 0], d[:steps, 1])
            if r["end"] != 1:
                continue
            ones = [int(out["sel"][s][g]) for g, v in zip(d[:steps, 0], d[:steps, 1]) if v == 1]
            assert all(r["e"][c] == 1 for c in ones), (s, p)
            assert r["pm"] >= sum(llr[c] for c in ones) * (1 - 1e-12), (s, p)
            checked += 1
    assert checked > 0


def test_path_bound_by_brute_force():
    """The path bound's lower bound against exhaustive search on tiny random
    instances: with VNs fixed to 1 (F1), fixed to 0, and the rest active (A),
    the cheapest answer meeting the syndrome that keeps the fixed values costs
    at least sum(F1) + [residual syndrome non-zero] * min(A); the bound is
    attained on some instances of both kinds, so a larger added term (the
    largest active prior, or the least one added while the residual syndrome
    is already met) fails."""
    rng = np.random.default_rng(17)
    tight_res, tight_zero, n_cases = 0, 0, 0
    for _ in range(400):
        m, n = int(rng.integers(2, 5)), int(rng.integers(3, 8))
        H = (rng.random((m, n)) < 0.5).astype(np.int64)
        prior = rng.uniform(0.5, 9.0, n)
        state = rng.integers(-1, 2, n)              # -1 active, 0 / 1 fixed
        act = np.nonzero(state < 0)[0]
        if act.size == 0:
            continue
        f1 = np.nonzero(state == 1)[0]
        e_true = rng.integers(0, 2, n)
        e_true[state >= 0] = state[state >= 0]        # consistent: an answer exists
        syn = H @ e_true % 2
        best = np.inf
        for mask in range(1 << act.size):
            e = (state == 1).astype(np.int64)
            e[act[[(mask >> j) & 1 == 1 for j in range(act.size)]]] = 1
            if ((H @ e) % 2 == syn).all():
                best = min(best, prior[e == 1].sum())
        res = (syn + H[:, f1].sum(axis=1)) % 2
        lower = prior[f1].sum() + (prior[act].min() if res.any() else 0.0)
        assert best >= lower - 1e-12
        n_cases += 1
        if abs(best - lower) <= 1e-12:
            if res.any():
                tight_res += 1
            else:
                tight_zero += 1
    assert n_cases > 300 and tight_res > 0 and tight_zero > 0


def test_unsatisfied_residual_adds_the_least_active_prior():
    """The second term of the path bound: at a step where the VNs a path has
    fixed to 1 (decimated or peeled) leave a non-zero residual syndrome, the
    path's answer, if it converges, sets at least one more VN, and only VNs
    still active can change; so its Eq. 5 metric is at least the fixed-to-1
    priors plus the least prior of the active VNs. Checked at every step of
    every converged path of the oracle's 16-path tree: the active VNs of a
    step are those with an Alg. 1 key, the fixed ones keep their value in the
    answer, and the residual syndrome is formed from the window matrix."""
    dem = circuit_dem(get_code("72"), 6, 0.004)
    prm = O.params(alpha=1.0, g=4, pre_iters=8, trunc_factor=2, low_error=1, dmax_main=25,
                   extra_steps=10)
    e = sample_errors(dem.thresholds(), 80, seed=5)
    det, _ = syndromes(dem, e)
    w = O.OracleWindow(dem, 0, 3)
    ex = w.export()
    H, llr = ex["H"].astype(np.int64), ex["llr"]
    syn = np.ascontiguousarray(det[:, w.row0:w.row0 + w.m])
    out = w.decode(prm, syn, logs=True)
    checked = tight = 0
    for s in range(syn.shape[0]):
        if out["ends"][s, :, 1].max() == 0:
            continue
        sel = out["sel"][s]
        for p in range(out["dec"].shape[1]):
            d = out["dec"][s, p]
            steps = int((d[:, 0] >= 0).sum())
            r = w.replay(prm, syn[s], sel, p, d[:steps, 0], d[:steps, 1])
            if r["end"] != 1:
                continue
            cols = sel[sel >= 0]
            for D in range(r["steps"]):
                keys = r["step_lsum"][D][:cols.size]
                if np.isnan(keys).all():
                    continue          # the step converged: no key recorded
                active = ~np.isnan(keys)
                fixed1 = cols[~active][r["e"][cols[~active]] == 1]
                res = (syn[s].astype(np.int64) + H[:, fixed1].sum(axis=1)) % 2
                lower = llr[fixed1].sum()
                if res.any():
                    lower += llr[cols[active]].min()
                    tight += 1
                assert r["pm"] >= lower * (1 - 1e-12), (s, p, D)
                checked += 1
    assert checked > 0 and tight > 0


@pytest.mark.parametrize("W,F", [(3, 1), (4, 1), (5, 2), (4, 3)])
def test_wf_windows_commit_every_column_once(W, F):
    """(W,F) sliding windows (Sec. III; App. E): window k holds rounds
    kF..kF+W-1, the last window is the first reaching the final round; every
    DEM column is committed by exactly one window, a window commits only
    columns no later window contains, and a column spilling past a non-last
    window's last round is replaced by unit columns there."""
    dem = circuit_dem(get_code("72"), 6, 0.003)
    K = O.n_windows(dem.n_rounds, W, F)
    assert (K - 2) * F + W < dem.n_rounds <= (K - 1) * F + W
    fr, lr = dem.first_round(), dem.last_round()
    count = np.zeros(dem.n_cols, int)
    later = [set() for _ in range(K)]
    exps = []
    for k in range(K):
        w = O.OracleWindow(dem, k, W, F)
        ex = w.export()
        exps.append(ex)
        r0 = k * F
        assert w.row0 == r0 * dem.w and w.m == min(W, dem.n_rounds - r0) * dem.w
        src = ex["src"]
        real = src >= 0
        for c in src[real & (ex["commit"] == 1)]:
            count[c] += 1
        last_round = r0 + w.m // dem.w - 1
        inside = np.nonzero((fr >= r0) & (fr <= last_round) & (lr <= last_round))[0]
        assert sorted(src[real].tolist()) == inside.tolist()
        for j in range(k):
            later[j] |= set(src[real].tolist())
    assert (count == 1).all()
    for k in range(K):
        src, com = exps[k]["src"], exps[k]["commit"]
        committed = set(src[(src >= 0) & (com == 1)].tolist())
        assert not committed & later[k]


def test_wf_commit_composes_to_eq8():
    """(5,2) windows on whole circuit-level shots: the residual detectors and
    observable accumulators the oracle reports equal H e + det and L e + obs
    recomputed here (Eq. 8, Eq. 9)."""
    dem = circuit_dem(get_code("72"), 6, 0.004)
    prm = O.params(alpha=1.0, g=4, pre_iters=8, trunc_factor=2, low_error=0)
    e = sample_errors(dem.thresholds(), 120, seed=13)
    det, obs = syndromes(dem, e)
    r = O.decode_shots(dem, 5, prm, det, obs, F=2)
    H = dem.dense_h().astype(np.int64)
    L = dem.dense_l().astype(np.int64)
    resid = (det.astype(np.int64) + r["e"].astype(np.int64) @ H.T) % 2
    assert np.array_equal(resid, r["det_out"])
    lres = (obs.astype(np.int64) + r["e"].astype(np.int64) @ L.T) % 2
    assert np.array_equal(lres, r["obs_out"])
    assert r["fail"].sum() < 120
    assert r["win_flags"].shape[1] == O.n_windows(dem.n_rounds, 5, 2)


def test_one_round_models_structure_and_decoding():
    """App. A and App. B problems: H is H_X (data noise) or [H_X | I] (single
    shot); the single-shot observables are the logical operators and H_X on
    the data columns. A single syndrome-bit flip is explained by its virtual
    column (a weight-one syndrome needs many data flips), a single data flip by
    its data column, and in both cases the correction counts as a success."""
    from gdg_inputs.dem import data_noise_dem, single_shot_dem
    code = get_code("72")
    dd = data_noise_dem(code, 0.03)
    assert np.array_equal(dd.dense_h(), code.hx) and dd.n_rounds == 1
    lg = logical_operators(code.hx, code.hz)
    assert np.array_equal(dd.dense_l(), lg)
    ss = single_shot_dem(code, 0.03, 0.001)
    m, n = code.hx.shape
    assert np.array_equal(ss.dense_h(), np.hstack([code.hx, np.eye(m, dtype=np.uint8)]))
    Lss = ss.dense_l()
    assert np.array_equal(Lss[:, :n], np.vstack([lg, code.hx])) and not Lss[:, n:].any()
    prm = O.params(alpha=0.625, g=4, low_error=1)
    for col in (n + 5, 17):
        e = np.zeros((1, ss.n_cols), np.uint8)
        e[0, col] = 1
        det, obs = syndromes(ss, e)
        r = O.decode_shots(ss, 1, prm, det, obs)
        assert r["fail"][0] == 0 and r["e"][0, col] == 1 and r["e"][0].sum() == 1


def _gf2_rank(M):
    M = (np.array(M, np.uint8) & 1).copy()
    r = 0
    rows, cols = M.shape
    for c in range(cols):
        piv = [i for i in range(r, rows) if M[i, c]]
        if not piv:
            continue
        M[[r, piv[0]]] = M[[piv[0], r]]
        for i in range(rows):
            if i != r and M[i, c]:
                M[i] ^= M[r]
        r += 1
    return r


@pytest.mark.parametrize("seed", range(8))
def test_osd_structure_and_exact_ml_on_small_problems(seed):
    """BP+OSD (Sec. II-A): with no BP iterations the ranking is the priors,
    ascending, ties by column. OSD-0's answer meets the syndrome and lies on
    the information set -- the first columns of that order that raise the GF(2)
    rank, found here by rank increments. With two non-pivot columns and
    lambda >= 2 the combination sweep tries every solution of H e = s, so its
    answer has the brute-force least Eq. 5 cost."""
    rng = np.random.default_rng(200 + seed)
    m, n = 7, 9
    while True:
        H = (rng.random((m, n)) < 0.4).astype(np.uint8)
        if _gf2_rank(H) == m:
            break
    llr = np.round(rng.uniform(0.5, 4.0, n), 1)          # ties among priors happen
    e0 = (rng.random(n) < 0.3).astype(np.uint8)
    syn = ((H.astype(int) @ e0) % 2).astype(np.uint8)
    prm = O.params(alpha=1.0)
    order = sorted(range(n), key=lambda c: (llr[c], c))
    S, cur = [], np.zeros((0, m), np.uint8)
    for c in order:
        nxt = np.vstack([cur, H[:, c][None, :]])
        if _gf2_rank(nxt) > len(S):
            S.append(c)
            cur = nxt
    pm0, e_0, fl0 = O.dense_osd(H, llr, syn, prm, n_iters=0, cs=False)
    assert fl0 == 1 and not (((H.astype(int) @ e_0) % 2) ^ syn).any()
    assert set(np.nonzero(e_0)[0]) <= set(S)
    assert abs(pm0 - float(llr @ e_0)) < 1e-12
    best = np.inf
    for bits in itertools.product([0, 1], repeat=n):
        e = np.array(bits)
        if not (((H.astype(int) @ e) % 2) ^ syn).any():
            best = min(best, float(llr @ e))
    pmc, e_c, flc = O.dense_osd(H, llr, syn, prm, n_iters=0, cs=True, lam=2)
    assert flc == 1 and not (((H.astype(int) @ e_c) % 2) ^ syn).any()
    assert abs(pmc - best) < 1e-9 and pmc <= pm0 + 1e-12


def test_osd_keeps_bp_answer_and_solves_windows():
    """When BP meets the syndrome, BP+OSD returns its hard decision; on
    circuit-level windows where it does not, OSD-CS10 on the whole window and
    on the first 2m ranked columns (Sec. III's shortening) both return answers
    that meet the window syndrome exactly."""
    dem = circuit_dem(get_code("72"), 6, 0.006)
    w = O.OracleWindow(dem, 1, 3)
    e = sample_errors(dem.thresholds(), 40, seed=17)
    det, obs = syndromes(dem, e)
    syn = np.ascontiguousarray(det[:, w.row0:w.row0 + w.m])
    H = w.export()["H"].astype(np.int64)
    prm = O.params(alpha=1.0)
    for n_keep in (0, 2 * w.m):
        r = w.osd(prm, syn, n_iters=30, cs=True, lam=10, n_keep=n_keep)
        osd_used = r["order"][:, 0] >= 0
        assert osd_used.any() and (~osd_used).any()
        for s in range(syn.shape[0]):
            if r["flags"][s] & 1:
                assert not ((H @ r["e"][s] + syn[s]) % 2).any()
        assert (r["flags"][~osd_used] & 1).all()
        assert (r["bp_iters"][osd_used] == 30).all()
        assert (r["flags"] & 1).mean() >= 0.95


def test_window_osd_pipeline_solves_every_window():
    """Sec. III's window comparator: the H1 block of each window before the
    last is merged into an identity, so its matrix has full row rank and
    BP+OSD on all kept columns solves it; once those are solved the last
    window's syndrome lies in its span too. So with OSD on every window each
    window flag says satisfied and the residual detectors end at zero. With
    OSD on the last window only (App. E), the earlier windows decode exactly as
    without it, and on shots whose GDG windows were all satisfied the last one
    is solved and its rows end clear."""
    dem = circuit_dem(get_code("72"), 6, 0.004)
    det, obs = syndromes(dem, sample_errors(dem.thresholds(), 24, seed=31))
    prm = O.params(alpha=1.0, g=4, pre_iters=8, trunc_factor=2, low_error=0)
    every = O.decode_shots(dem, 3, prm, det, obs, osd=(60, 10, 0), osd_on="all")
    assert (every["win_flags"] & 1).all()
    assert not every["det_out"].any()
    base = O.decode_shots(dem, 3, prm, det, obs)
    last = O.decode_shots(dem, 3, prm, det, obs, osd=(60, 10, 0))
    assert np.array_equal(last["win_flags"][:, :-1], base["win_flags"][:, :-1])
    assert (base["win_flags"] & 1).all()   # so the last window's syndrome is in its span
    assert (last["win_flags"][:, -1] & 1).all()
    K = O.n_windows(dem.n_rounds, 3, 1)
    assert not last["det_out"][:, O.OracleWindow(dem, K - 1, 3).row0:].any()


def test_warm_start_hand_example():
    """Warm start (reading of Sec. V's message reuse) on a hand-computed
    example: the carried CN-to-VN message enters through one VN update before
    the first iteration (it changes VN2's posterior through VN1's extrinsic
    message), and the hand-over is one CN update of the final VN-to-CN
    messages (not the last CN messages themselves, which are [-3, -2, 4, -2])."""
    warm, cold = _read_cases("warm_start_2cn_3vn.txt")
    prm = O.params(alpha=1.0, pre_iters=4, trunc_factor=2)
    for case, wi in ((warm, warm.get("warm_in")), (cold, None)):
        r = O.dense_window(case["H"], case["llr"], case["syn"].astype(np.uint8), prm,
                           warm_in=wi, warm_out=True)
        np.testing.assert_allclose(r["lsum"], case["lsum"], rtol=0, atol=1e-15)
        np.testing.assert_allclose(r["warm_out"], case["warm_out"], rtol=0, atol=1e-15)
        assert r["e"].tolist() == case["ehat"].astype(int).tolist()
        assert r["pm"] == case["pm"][0] and r["flags"] & 1


def test_warm_zero_messages_equal_cold_start():
    """Carried messages that are all zero leave the window decode exactly as
    the cold start (the VN update then forms the priors' messages)."""
    dem = circuit_dem(get_code("72"), 6, 0.004)
    det, obs = syndromes(dem, sample_errors(dem.thresholds(), 40, seed=43))
    w = O.OracleWindow(dem, 2, 3)
    prm = O.params(alpha=1.0, g=4, pre_iters=8, trunc_factor=2, low_error=0)
    syn = np.ascontiguousarray(det[:, w.row0:w.row0 + w.m])
    cold = w.decode(prm, syn, warm_out=True)
    zero = w.decode(prm, syn, warm_in=np.zeros((syn.shape[0], w.n_edges)), warm_out=True)
    for k in ("e", "flags", "edge_iters"):
        assert np.array_equal(cold[k], zero[k]), k
    assert np.array_equal(cold["pm"], zero["pm"])
    assert np.array_equal(cold["warm_out"], zero["warm_out"])


def test_warm_map_joins_the_same_row_and_column():
    """The edge map between consecutive windows (1..4 of (3,1), and (5,2)):
    every mapped pair is the same detector row and DEM column, and every edge
    of the next window whose DEM column and row the previous window also has
    is mapped (brute force over the dense window matrices); unit columns
    never are."""
    dem = circuit_dem(get_code("72"), 8, 0.003)
    for W, F, ks in ((3, 1, (1, 2, 5)), (5, 2, (1, 2))):
        for k in ks:
            a, b = O.OracleWindow(dem, k - 1, W, F), O.OracleWindow(dem, k, W, F)
            ea, eb = a.export(), b.export()
            mp = b.warm_map(a)
            ra, ca = np.nonzero(ea["H"])      # row-major edge order
            rb, cb = np.nonzero(eb["H"])
            assert len(mp) == len(rb)
            key_a = {(a.row0 + r, ea["src"][c]): i for i, (r, c) in enumerate(zip(ra, ca))
                     if ea["src"][c] >= 0}
            n_mapped = 0
            for i, (r, c) in enumerate(zip(rb, cb)):
                want = key_a.get((b.row0 + r, eb["src"][c])) if eb["src"][c] >= 0 else None
                if want is None:
                    assert mp[i] == -1, (W, F, k, i)
                else:
                    assert mp[i] == want, (W, F, k, i)
                    n_mapped += 1
            assert n_mapped > 0
