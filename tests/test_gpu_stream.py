"""Streaming service on the GPU: every experiment it finishes decodes exactly
as the offline sliding-window decoder decodes the same shot (same window
results, commits into per-block records at their own offsets), across codes,
window shapes and batch compositions; admission control rejects what does not
fit."""
import numpy as np
import pytest

from gdg_inputs.bb import get_code
from gdg_inputs.dem import circuit_dem

torch = pytest.importorskip("torch")
gpu = pytest.mark.gpu


def _mods():
    import paper_2403_18901_amd.gdg as G
    import paper_2403_18901_amd.stream as S
    return G, S


def _offline(G, c, prm, ids):
    n = int(ids.max()) + 1
    det, obs = c.ddem.sample(n, seed=c.seed, stream=c.stream_id, shot0=0)
    fail, _ = G.SlidingWindowDecoder(c.dem, prm).decode(det, obs)
    return fail.cpu().numpy(), obs.cpu().numpy()


@gpu
def test_stream_matches_offline_decoder():
    G, S = _mods()
    p = 0.003
    prm = G.params(alpha=1.0, g=4, pre_iters=8, trunc_factor=2, low_error=0)
    codes = [(circuit_dem(get_code("72"), 6, p), 6), (circuit_dem(get_code("144"), 4, p), 3)]
    svc = S.StreamingService(codes, prm, rate=500.0, n_slots=64, seed=11)
    rep = svc.run(duration=0.15)
    assert rep["rejected"] == 0 and rep["windows"] > 0
    for c in svc.codes:
        assert len(c.fails) >= 10
        ids = np.array([e for e, _ in c.fails])
        f_off, o_off = _offline(G, c, prm, ids)
        for e, f in c.fails:
            assert f == f_off[e], e
            assert np.array_equal(c.obs_out[e], o_off[e]), e
    assert rep["latency_ms"]["p50"] > 0


@gpu
def test_stream_admission_rejects_over_budget():
    G, S = _mods()
    prm = G.params(alpha=1.0, g=4, pre_iters=8, trunc_factor=2, low_error=1)
    codes = [(circuit_dem(get_code("72"), 6, 0.002), 8)]
    svc = S.StreamingService(codes, prm, rate=1e5, n_slots=4, seed=5)
    rep = svc.run(duration=0.01)
    assert rep["rejected"] > 0
    assert rep["admitted"] + rep["rejected"] == rep["experiments_started"]
    c = svc.codes[0]
    ids = np.array([e for e, _ in c.fails])
    f_off, o_off = _offline(G, c, prm, ids)
    for e, f in c.fails:
        assert f == f_off[e] and np.array_equal(c.obs_out[e], o_off[e])
