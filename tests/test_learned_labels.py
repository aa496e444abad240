"""CPU: the learned proposer's training labels for unit columns. A window's
unit column merges the columns that start inside the window and reach past
its last round, one unit column per last-round row they touch (Sec. III);
its label is the parity of those columns' errors on that row. The merged
set the training code finds is pinned by the oracle's own merge: the unit
column's prior equals (1 - prod(1 - 2 p_c)) / 2 over exactly those columns."""
import numpy as np
import pytest

from gdg_inputs.bb import get_code
from gdg_inputs.dem import circuit_dem
from oracle import oracle as O


def _lrn():
    import paper_2403_18901_amd.learned as L
    return L


@pytest.mark.parametrize("key,rounds,k", [("72", 6, 0), ("144", 12, 0), ("144", 12, 5)])
def test_unit_column_sources_reproduce_the_merged_priors(key, rounds, k):
    dem = circuit_dem(get_code(key), rounds, 0.003)
    ow = O.OracleWindow(dem, k, 3)
    ex = ow.export()
    units = _lrn().unit_column_sources(dem, ex["src"], ow.row0)
    unit_idx = np.nonzero(ex["src"] < 0)[0]
    assert len(units) == unit_idx.size > 0
    pri = np.asarray(dem.priors, np.float64)
    for j in unit_idx:
        r = int(-1 - ex["src"][j])
        cols = units[r]
        assert cols.size > 0
        assert ow.row0 + r in set().union(*[set(dem.col_rows(c).tolist()) for c in cols])
        merged = 0.5 * (1.0 - np.prod(1.0 - 2.0 * pri[cols]))
        assert ex["prior"][j] == pytest.approx(merged, rel=1e-12), (j, r)


def test_unit_label_is_the_parity_on_the_row():
    """On sampled errors, a unit column's label equals the row's syndrome bit
    minus the window columns' contribution, over the columns that started in
    the window (earlier columns excluded), i.e. what a correct correction
    would set it to."""
    dem = circuit_dem(get_code("72"), 6, 0.004)
    ow = O.OracleWindow(dem, 0, 3)
    ex = ow.export()
    units = _lrn().unit_column_sources(dem, ex["src"], ow.row0)
    H = dem.dense_h().astype(np.int64)
    rng = np.random.default_rng(3)
    e = (rng.random((50, dem.n_cols)) < 0.02).astype(np.int64)
    own = ex["src"][ex["src"] >= 0]
    first = dem.first_round()
    for r, cols in units.items():
        row = ow.row0 + r
        later = np.nonzero((first >= ow.row0 // dem.w) & (H[row] == 1))[0]
        outside = np.setdiff1d(later, own)
        np.testing.assert_array_equal(np.sort(outside), np.sort(cols))
        label = e[:, cols].sum(1) % 2
        rest = e[:, np.intersect1d(later, own)].sum(1) % 2
        np.testing.assert_array_equal((label + rest) % 2, (e[:, later] @ np.ones(later.size, np.int64)) % 2)
