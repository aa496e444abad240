"""CPU: the grouping and launch shapes of batched.LaunchPlan (the device call
is replaced by a recorder; no GPU is needed)."""
import pytest


class _Win:
    def __init__(self, n_act):
        self.n_act = n_act


def _record(monkeypatch):
    import paper_2403_18901_amd.batched as B
    calls = []
    monkeypatch.setattr(B.G, "decode_jobs",
                        lambda grp, waves, workgroups: calls.append(
                            ([j[0].n_act for j in grp], waves, workgroups)))
    return B, calls


def test_one_launch_when_not_split(monkeypatch):
    B, calls = _record(monkeypatch)
    jobs = [(_Win(864), 0, 0, None), (_Win(432), 0, 0, None), (_Win(216), 0, 0, None)]
    B.LaunchPlan(waves=8, wg_per_cu=2).run(jobs)
    assert calls == [([864, 432, 216], 8, 2 * B.N_CU)]


def test_split_launches_per_tiling_with_their_own_shapes(monkeypatch):
    B, calls = _record(monkeypatch)
    jobs = [(_Win(864), 0, 0, None), (_Win(432), 0, 0, None), (_Win(270), 0, 0, None),
            (_Win(216), 0, 0, None)]
    plan = B.LaunchPlan(waves=4, split=True, per_bucket={3: (8, 2), 0: (2, 0)})
    plan.run(jobs)
    # largest tiling first; a tiling without an entry takes the plan's shape
    assert calls == [([864], 8, 2 * B.N_CU), ([432], 4, 0), ([270, 216], 2, 0)]
    assert plan.key() != B.LaunchPlan(waves=4, split=True).key()
    assert B.LaunchPlan(waves=4, per_bucket={3: (8, 2)}).per_bucket == {}   # split only


@pytest.mark.parametrize("n_act,bucket", [(216, 0), (384, 0), (432, 1), (448, 1), (512, 2),
                                          (864, 3), (896, 3), (1000, 4)])
def test_tiling_buckets(n_act, bucket):
    import paper_2403_18901_amd.batched as B
    assert B._bucket(_Win(n_act)) == bucket
