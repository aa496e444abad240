"""BP + OSD-CS on the GPU (gdg_decode_osd) against the oracle.

The GPU ranks columns by FP32 posteriors and the oracle by FP64 ones, so
near-equal posteriors may be ordered differently; everything after the
ranking (elimination, the combination sweep, the Eq. 5 costs in double) is
exact for a given order. The checks: the GPU's order is the ascending, ties
by column, order of its own BP posteriors after the same iterations (gdg_bp);
the oracle handed the GPU's order reproduces answer, metric and flags bit for
bit; BP convergence agrees with the oracle's on nearly every shot; and whole
sliding-window decodes with BP+OSD windows fail on the oracle's shots within
the oracle's 2-sigma interval.
"""
import numpy as np
import pytest

from gdg_inputs.bb import get_code
from gdg_inputs.dem import circuit_dem
from gdg_inputs.philox import sample_errors, syndromes
from oracle import oracle as O
from test_gpu_parity import _residual_before, wilson

torch = pytest.importorskip("torch")
gpu = pytest.mark.gpu

BP_ITERS = 200   # the window BP+OSD-CS10 of Fig. 3's comparator


def _gdg():
    import paper_2403_18901_amd.gdg as G
    return G


def _prm(G, p):
    return G.params(alpha=1.0, g=4, pre_iters=8, trunc_factor=2, low_error=int(p <= 0.002))


def _oprm(p):
    return O.params(alpha=1.0, g=4, pre_iters=8, trunc_factor=2, low_error=int(p <= 0.002))


def _valid_ranking(post, order):
    """order is a permutation of the columns that sorts post ascending, equal
    values by ascending column (-0.0 counts below +0.0, as in the key)."""
    n = post.shape[0]
    assert np.array_equal(np.sort(order), np.arange(n))
    v = post[order]
    assert (np.diff(v) >= 0).all()
    same = v[1:] == v[:-1]
    same_sign = np.signbit(v[1:]) == np.signbit(v[:-1])
    assert (np.diff(order)[same & same_sign] > 0).all()


@gpu
@pytest.mark.parametrize("key,rounds,p,k,n_keep", [
    ("72", 6, 0.006, 1, 0),
    ("72", 6, 0.006, 1, -2),
    ("144", 6, 0.004, 1, 0),
    ("144", 6, 0.004, 1, -2),
    ("144", 6, 0.003, 0, -2),
    ("288", 4, 0.004, 1, -2),
])
def test_osd_window_replays_bit_exact(key, rounds, p, k, n_keep):
    G = _gdg()
    dem = circuit_dem(get_code(key), rounds, p)
    e = sample_errors(dem.thresholds(), 96, seed=61)
    det, obs = syndromes(dem, e)
    det = _residual_before(dem, _oprm(p), det, obs, k)
    w = G.Window(dem, k, 3, _prm(G, p))
    ow = O.OracleWindow(dem, k, 3)
    nk = 2 * w.m if n_keep == -2 else n_keep
    d = torch.from_numpy(det).cuda()
    print(f"osd replay {key} p={p} k={k} n_keep={nk} shots={det.shape[0]}", flush=True)
    eg, pmg, flg, ordg, itg = w.decode_osd(d, syn_offset=w.row0, bp_iters=BP_ITERS, cs=True,
                                           lam=10, n_keep=nk, trace=True)
    torch.cuda.synchronize()
    eg, pmg, flg = eg.cpu().numpy(), pmg.cpu().numpy(), flg.cpu().numpy()
    ordg, itg = ordg.cpu().numpy(), itg.cpu().numpy()
    syn = np.ascontiguousarray(det[:, w.row0:w.row0 + w.m])
    H = ow.export()["H"].astype(np.int64)

    # every satisfied answer meets the window syndrome; the full-column OSD always does
    for s in range(syn.shape[0]):
        if flg[s] & 1:
            assert not ((H @ eg[s] + syn[s]) % 2).any(), s
            assert np.isfinite(pmg[s])
        else:
            assert np.isinf(pmg[s])
    if nk == 0:
        assert (flg & 1).all()

    ref = ow.osd(_oprm(p), syn, n_iters=BP_ITERS, cs=True, lam=10, n_keep=nk)
    g_osd = ordg[:, 0] >= 0
    o_osd = ref["order"][:, 0] >= 0
    assert (itg[g_osd] == BP_ITERS).all()
    assert ((itg[~g_osd] >= 1) & (itg[~g_osd] <= BP_ITERS)).all()
    both_bp = ~g_osd & ~o_osd
    if both_bp.any():
        assert (itg[both_bp] == ref["bp_iters"][both_bp]).mean() >= 0.9
    agree = (g_osd == o_osd).mean()
    print(f"OSD used on {g_osd.sum()} GPU / {o_osd.sum()} oracle shots; agree {agree:.3f}")
    assert agree >= 0.95
    assert g_osd.sum() >= 10   # the case exercises the elimination
    # BP answers where both converged: the same hard decision on nearly all shots
    if both_bp.any():
        assert (eg[both_bp] == ref["e"][both_bp]).all(axis=1).mean() >= 0.9

    # the GPU's ranking is the stable ascending order of its own posteriors
    idx = np.nonzero(g_osd)[0]
    post, first = w.bp(d[torch.from_numpy(idx).cuda()], BP_ITERS, syn_offset=w.row0)
    torch.cuda.synchronize()
    last = post[:, BP_ITERS - 1, :].cpu().numpy()
    assert (first.cpu().numpy() == 0).all()
    for r, s in enumerate(idx):
        _valid_ranking(last[r], ordg[s])

    # the oracle, handed the GPU's order, reproduces the answer bit for bit
    rep = idx[o_osd[idx]]
    fo = np.ascontiguousarray(ordg[rep])
    rr = ow.osd(_oprm(p), syn[rep], n_iters=BP_ITERS, cs=True, lam=10, n_keep=nk,
                forced_order=fo)
    assert np.array_equal(rr["order"], fo)
    assert np.array_equal(rr["e"], eg[rep])
    assert np.array_equal(rr["flags"], flg[rep])
    assert np.array_equal(rr["pm"].view(np.uint64), pmg[rep].view(np.uint64))


@gpu
def test_osd_kernel_edge_cases():
    """Zero syndromes converge at the first iteration with the empty answer;
    OSD-0 (cs off) and lambda 0 or 1 (no pairs) run; an all-shots-empty call
    is a no-op; shapes beyond the kernel's limits are refused."""
    G = _gdg()
    p = 0.004
    dem = circuit_dem(get_code("72"), 6, p)
    det, obs = syndromes(dem, sample_errors(dem.thresholds(), 40, seed=62))
    w = G.Window(dem, 1, 3, _prm(G, p))
    ow = O.OracleWindow(dem, 1, 3)
    z = torch.zeros((4, det.shape[1]), dtype=torch.uint8, device="cuda")
    e0, pm0, fl0, ord0, it0 = w.decode_osd(z, syn_offset=w.row0, bp_iters=5, trace=True)
    torch.cuda.synchronize()
    assert not e0.any() and (pm0 == 0).all() and (fl0 == 1).all()
    assert (ord0 == -1).all() and (it0 == 1).all()
    d = torch.from_numpy(det).cuda()
    syn = np.ascontiguousarray(det[:, w.row0:w.row0 + w.m])
    for cs, lam in ((False, 10), (True, 0), (True, 1), (True, 3)):
        eg, pmg, flg, ordg, _ = w.decode_osd(d, syn_offset=w.row0, bp_iters=30, cs=cs, lam=lam,
                                             trace=True)
        torch.cuda.synchronize()
        eg, pmg, flg, ordg = (t.cpu().numpy() for t in (eg, pmg, flg, ordg))
        ref = ow.osd(_oprm(p), syn, n_iters=30, cs=cs, lam=lam)
        rep = np.nonzero((ordg[:, 0] >= 0) & (ref["order"][:, 0] >= 0))[0]
        assert len(rep) >= 10
        rr = ow.osd(_oprm(p), syn[rep], n_iters=30, cs=cs, lam=lam,
                    forced_order=np.ascontiguousarray(ordg[rep]))
        assert np.array_equal(rr["e"], eg[rep]), (cs, lam)
        assert np.array_equal(rr["pm"].view(np.uint64), pmg[rep].view(np.uint64)), (cs, lam)
        assert np.array_equal(rr["flags"], flg[rep])
    empty = torch.zeros((0, det.shape[1]), dtype=torch.uint8, device="cuda")
    out = w.decode_osd(empty, syn_offset=w.row0, bp_iters=5)
    assert out[0].shape[0] == 0
    big = G.Window(circuit_dem(get_code("288"), 4, p), 1, 3, _prm(G, p))
    zb = torch.zeros((1, big.row0 + big.m), dtype=torch.uint8, device="cuda")
    with pytest.raises(RuntimeError):
        big.decode_osd(zb, syn_offset=big.row0, bp_iters=5)   # all 3456 columns: LDS
    big.decode_osd(zb, syn_offset=big.row0, bp_iters=5, n_keep=2 * big.m)


@gpu
@pytest.mark.parametrize("osd_on", ["all", "last"])
def test_sliding_window_osd_ler_parity(osd_on):
    """(3,1) sliding windows with BP(200)+OSD-CS10 on every window (Fig. 3's
    window comparator) or on the last window only (App. E): failures within
    the oracle's 2-sigma interval on the same shots, and the same window
    verdicts as the oracle on nearly every shot."""
    G = _gdg()
    p = 0.004
    dem = circuit_dem(get_code("72"), 6, p)
    det, obs = syndromes(dem, sample_errors(dem.thresholds(), 400, seed=63))
    osd = (BP_ITERS, 10, 0)
    dec = G.SlidingWindowDecoder(dem, _prm(G, p), W=3, osd=osd, osd_on=osd_on)
    d = torch.from_numpy(det).cuda()
    o = torch.from_numpy(obs).cuda()
    print(f"sliding window osd_on={osd_on} shots={det.shape[0]}", flush=True)
    fail, wflags = dec.decode(d, o)
    torch.cuda.synchronize()
    gf = fail.cpu().numpy().astype(bool)
    res = d.cpu().numpy()
    wf = wflags.cpu().numpy()
    # where every earlier window was satisfied, OSD solves the last one and
    # every row ends clear (after a failed window the residual can leave the
    # last window's span)
    ok_before = (wf[:, :-1] & 1).all(axis=1)
    assert ok_before.mean() >= 0.9
    assert (wf[ok_before, -1] & 1).all()
    assert not res[(wf & 1).all(axis=1)].any()
    assert not res[wf[:, -1] & 1 == 1][:, dec.windows[-1].row0:].any()
    ref = O.decode_shots(dem, 3, _oprm(p), det, obs, osd=osd, osd_on=osd_on)
    nf = int(ref["fail"].sum())
    lo, hi = wilson(nf, len(gf))
    print(f"failures GPU {int(gf.sum())}, oracle {nf} of {len(gf)}; "
          f"same verdict on {(gf == ref['fail'].astype(bool)).mean():.3f}")
    assert lo * len(gf) - 1e-9 <= gf.sum() <= hi * len(gf) + 1e-9
    assert (gf == ref["fail"].astype(bool)).mean() >= 0.95
