"""gdg_decode_batch with a caller workspace (no allocation, no
synchronisation inside the call) against the library's own scratch pool:
identical answers with a workspace of gdg_workspace_bytes, and with one that
holds the counter and a single workgroup's checkpoints (the other workgroups
then replay their paths from the root). Bad workspaces are refused."""
import numpy as np
import pytest

from gdg_inputs.bb import get_code
from gdg_inputs.dem import circuit_dem
from gdg_inputs.philox import sample_errors, syndromes

torch = pytest.importorskip("torch")
gpu = pytest.mark.gpu


@gpu
def test_workspace_decode_matches_pool():
    import paper_2403_18901_amd.gdg as g
    p = 0.003
    dem = circuit_dem(get_code("144"), 12, p)
    prm = g.params(alpha=1.0, g=4, pre_iters=8, trunc_factor=2, low_error=0)
    w = g.Window(dem, 4, 3, prm)
    det, _ = syndromes(dem, sample_errors(dem.thresholds(), 4000, seed=43))
    d = torch.from_numpy(det).cuda()
    ref = w.decode(d, syn_offset=w.row0)
    full = w.workspace_bytes(d.shape[0])
    per_wg = (full - 256) // min(d.shape[0], 768) if full > 256 else 0
    assert full > 256 and per_wg > 0
    for nbytes in (full, 256 + per_wg, 256):
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        out = (torch.empty_like(ref[0]), torch.empty_like(ref[1]), torch.empty_like(ref[2]))
        w.decode_into(d, w.row0, out, workspace=ws)
        torch.cuda.synchronize()
        assert torch.equal(out[0], ref[0]), nbytes
        assert torch.equal(out[1].view(torch.int64), ref[1].view(torch.int64)), nbytes
        assert torch.equal(out[2], ref[2]), nbytes
    small = torch.empty(128, dtype=torch.uint8, device="cuda")
    with pytest.raises(RuntimeError):
        w.decode_into(d, w.row0, (torch.empty_like(ref[0]), torch.empty_like(ref[1]),
                                  torch.empty_like(ref[2])), workspace=small)
    g.release_scratch()
    again = w.decode(d, syn_offset=w.row0)
    torch.cuda.synchronize()
    assert torch.equal(again[0], ref[0])
