"""Cross-window message reuse (warm start) on the GPU against the oracle.

The GPU hands over FP32 messages and the oracle FP64 ones, so the checks
follow the posterior bars: the messages a window hands over agree with the
oracle's within 1e-4 relative (sign ties aside) on shots whose preprocessing
ran the same iterations; the next window, started on both sides from the
GPU's handed-over messages, decodes to the same answers and decisions as the
oracle (the window comparator's bars); whole warm-started shots fail inside
the oracle's 2-sigma interval; and a call that only hands over messages
decodes exactly as the cold decode.
"""
import numpy as np
import pytest

from gdg_inputs.bb import get_code
from gdg_inputs.dem import circuit_dem
from gdg_inputs.philox import sample_errors, syndromes
from oracle import oracle as O
from test_gpu_parity import _compare_window, _residual_before, wilson

torch = pytest.importorskip("torch")
gpu = pytest.mark.gpu


def _gdg():
    import paper_2403_18901_amd.gdg as G
    return G


def _prm(G, p):
    return G.params(alpha=1.0, g=4, pre_iters=8, trunc_factor=2, low_error=int(p <= 0.002))


def _oprm(p):
    return O.params(alpha=1.0, g=4, pre_iters=8, trunc_factor=2, low_error=int(p <= 0.002))


def _setup(p, k, ns, seed):
    dem = circuit_dem(get_code("144"), 12, p)
    det, obs = syndromes(dem, sample_errors(dem.thresholds(), ns, seed=seed))
    det = _residual_before(dem, _oprm(p), det, obs, k)
    return dem, det


def _gpu_pre_iters(tr, pre_iters):
    """Preprocessing iterations the GPU ran per shot (the trace's posteriors
    are NaN for iterations not run)."""
    pp = tr["pre_post"].cpu().numpy()
    return pre_iters - np.isnan(pp[:, :, 0]).sum(axis=1)


@gpu
@pytest.mark.parametrize("p,k", [(0.002, 3), (0.003, 5)])
def test_handed_over_messages_match_oracle(p, k):
    G = _gdg()
    dem, det = _setup(p, k, 120, 71)
    w = G.Window(dem, k, 3, _prm(G, p))
    ow = O.OracleWindow(dem, k, 3)
    d = torch.from_numpy(det).cuda()
    wout = torch.full((det.shape[0], w.n_msg), float("nan"), dtype=torch.float32, device="cuda")
    print(f"hand-over p={p} k={k}", flush=True)
    _, _, _, tr = w.decode(d, syn_offset=w.row0, trace=True, pre_post=True, warm_out=wout)
    torch.cuda.synchronize()
    g_iters = _gpu_pre_iters(tr, 8)
    g_conv = tr["sel"].cpu().numpy()[:, 0] < 0
    syn = np.ascontiguousarray(det[:, w.row0:w.row0 + w.m])
    ref = ow.decode(_oprm(p), syn, logs=True, warm_out=True)
    o_conv = ref["pre_converged"].astype(bool)
    o_iters = np.where(o_conv, ref["bp_iters"], 8)
    slots = w.edge_slots()
    g_msgs = wout.cpu().numpy()[:, slots].astype(np.float64)
    same = (g_conv == o_conv) & (g_iters == o_iters)
    assert same.mean() >= 0.95
    ties = 0
    for s in np.nonzero(same)[0]:
        a, b = g_msgs[s], ref["warm_out"][s]
        ok = np.abs(a - b) <= 1e-4 * np.maximum(1.0, np.abs(b))
        # a VN-to-CN message within 1e-3 of zero may take either sign in FP32:
        # the CN messages it feeds are then that small too
        ok |= np.abs(b) <= 1e-3
        if not ok.all():
            ties += 1
        assert ok.mean() >= 0.999, s
    assert ties <= max(2, same.sum() // 20)


@gpu
@pytest.mark.parametrize("p,k", [(0.002, 4), (0.003, 6)])
def test_warm_window_matches_oracle(p, k):
    """Window k decoded on both sides from the messages the GPU's window k-1
    handed over (the oracle gets them per edge, through its own edge map):
    answers, metrics and decisions to the window comparator's bars, and the
    preprocessing posteriors of the warm start within 1e-4."""
    G = _gdg()
    dem, det = _setup(p, k - 1, 160, 73)
    prev = G.Window(dem, k - 1, 3, _prm(G, p))
    w = G.Window(dem, k, 3, _prm(G, p))
    w.link(prev)
    d = torch.from_numpy(det).cuda()
    ns = det.shape[0]
    buf = torch.empty((ns, prev.n_msg), dtype=torch.float32, device="cuda")
    print(f"warm window p={p} k={k}", flush=True)
    e, _, _ = prev.decode(d, syn_offset=prev.row0, warm_out=buf)
    o = torch.zeros((ns, dem.n_obs), dtype=torch.uint8, device="cuda")
    prev.commit(e, d, o)
    torch.cuda.synchronize()
    det_k = d.cpu().numpy()
    # the same messages per edge of window k in the oracle's order
    ow, owp = O.OracleWindow(dem, k, 3), O.OracleWindow(dem, k - 1, 3)
    mp = ow.warm_map(owp)
    pslots = prev.edge_slots()
    g_prev = buf.cpu().numpy().astype(np.float64)
    o_in = np.full((ns, ow.n_edges), np.nan)
    o_in[:, mp >= 0] = g_prev[:, pslots[mp[mp >= 0]]]
    assert (mp >= 0).sum() > ow.n_edges // 3
    # posteriors of the warm-started preprocessing against the oracle's
    _, _, _, tr = w.decode(d, syn_offset=w.row0, trace=True, pre_post=True, warm_in=buf)
    torch.cuda.synchronize()
    pp = tr["pre_post"].cpu().numpy()
    syn = np.ascontiguousarray(det_k[:, w.row0:w.row0 + w.m])
    n_tie = 0
    for s in range(min(ns, 60)):
        post, _, cmin = ow.bp(_oprm(p), syn[s], 8, with_cn_min=True, warm_in=o_in[s])
        ran = int((~np.isnan(pp[s][:, 0])).sum())
        assert ran >= 1
        for t in range(ran):
            ok = np.abs(pp[s][t] - post[t]) <= 1e-4 * np.maximum(1.0, np.abs(post[t]))
            if not ok.all():
                # the posterior bar's sign-tie exception: a VN next to a CN whose
                # smallest incoming message is within 1e-3 of zero
                assert (cmin[t] <= 1e-3).any(), (s, t)
                n_tie += 1
                break
    assert n_tie <= 6
    _compare_window(dem, k, _prm(G, p), _oprm(p), det_k, require_exact=0.98,
                    warm=(buf, o_in), window=w)


@gpu
def test_hand_over_only_changes_nothing_and_errors():
    """A decode that only hands over messages gives the cold decode's answers,
    metrics and flags bit for bit; warm input on an unlinked window and warm
    buffers on a window without preprocessing are refused."""
    G = _gdg()
    p = 0.003
    dem, det = _setup(p, 2, 600, 75)
    w = G.Window(dem, 2, 3, _prm(G, p))
    d = torch.from_numpy(det).cuda()
    cold = w.decode(d, syn_offset=w.row0)
    buf = torch.empty((det.shape[0], w.n_msg), dtype=torch.float32, device="cuda")
    warm = w.decode(d, syn_offset=w.row0, warm_out=buf)
    torch.cuda.synchronize()
    assert torch.equal(cold[0], warm[0])
    assert torch.equal(cold[1].view(torch.int64), warm[1].view(torch.int64))
    assert torch.equal(cold[2], warm[2])
    assert torch.isfinite(buf).all()
    with pytest.raises(RuntimeError):
        w.decode(d, syn_offset=w.row0, warm_in=buf)          # not linked
    # plain BPGD on a phenomenological window: no preprocessing BP to warm-start
    from gdg_inputs.dem import phenomenological_dem
    dem0 = phenomenological_dem(get_code("72"), 6, 0.005, 0.005)
    w0 = G.Window(dem0, 2, 3, G.params(alpha=0.625, g=0, pre_iters=0, low_error=1))
    d0 = torch.zeros((4, dem0.n_rows), dtype=torch.uint8, device="cuda")
    b0 = torch.empty((4, max(1, w0.n_msg)), dtype=torch.float32, device="cuda")
    with pytest.raises(RuntimeError):
        w0.decode(d0, syn_offset=w0.row0, warm_out=b0)


@gpu
@pytest.mark.parametrize("p,ns", [(0.003, 20000), (0.002, 20000)])
def test_warm_pipeline_ler_parity(p, ns):
    """Whole 12-round shots with every window warm-started from the previous
    one: failures inside the oracle's 2-sigma interval (the oracle warm-starts
    the same way in FP64), zero residual detectors on every GPU success, and
    the failure counts of warm and cold decoding reported side by side."""
    G = _gdg()
    dem = circuit_dem(get_code("144"), 12, p)
    det, obs = syndromes(dem, sample_errors(dem.thresholds(), ns, seed=77))
    dec = G.SlidingWindowDecoder(dem, _prm(G, p), W=3, warm=True)
    d = torch.from_numpy(det).cuda()
    o = torch.from_numpy(obs).cuda()
    print(f"warm pipeline p={p} shots={ns}", flush=True)
    fail, _ = dec.decode(d, o)
    torch.cuda.synchronize()
    gf = fail.cpu().numpy().astype(bool)
    assert not d.cpu().numpy()[~gf].any()
    ref = O.decode_shots(dem, 3, _oprm(p), det, obs, warm=True)
    cold = O.decode_shots(dem, 3, _oprm(p), det, obs)
    rf = ref["fail"].astype(bool)
    lo, hi = wilson(int(rf.sum()), ns)
    print(f"p={p}: GPU warm failures {int(gf.sum())}, oracle warm {int(rf.sum())}, "
          f"oracle cold {int(cold['fail'].sum())} of {ns}; edge-iterations warm "
          f"{ref['edge_iters']} cold {cold['edge_iters']}")
    assert lo * ns - 1e-9 <= gf.sum() <= hi * ns + 1e-9
    assert (gf == rf).mean() >= 0.995
