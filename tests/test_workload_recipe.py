"""The synthetic workloads are shaped like the paper's graphs (Section 5,
Table 1; values in tests/golden/paper_table1_graphs.txt): vertex and edge
counts of the same size class, and the same directedness.  The non-zero
counts are those the seeded generator produces at full size (measured once;
the full-size GPU tests and the benchmark assert them again)."""
import os

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_table1_graphs.txt")

# (paper graph, scale, edge factor, symmetrised, non-zeros the generator gives)
STAND_INS = [("Twitter", 25, 44, False, 1431381365), ("Friendster", 26, 28, True, 3647439224)]


def _table():
    rows = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, v, e, d = line.split()
        rows[name] = (float(v), float(e), d)
    return rows


def test_stand_ins_match_table_1():
    t = _table()
    assert set(t) == {"Twitter", "Friendster", "Page", "RMAT-40", "RMAT-160"}
    for name, scale, ef, sym, nnz in STAND_INS:
        v, e, d = t[name]
        n = 1 << scale
        edges = nnz / 2 if sym else nnz              # a symmetrised edge is stored twice
        assert 0.75 <= n / v <= 1.25, name
        assert 0.9 <= edges / e <= 1.1, name
        assert (d == "undirected") == sym, name
        # the nominal edge count before duplicate removal is scale-free: 2^scale * ef
        assert nnz <= (2 if sym else 1) * n * ef


def test_generator_dedup_ratio_trend_reaches_the_full_size_counts():
    """The full-size non-zero counts above come from the same generator whose
    duplicate-removal ratio is checked here at small scales: the kept
    fraction of the drawn edges rises with scale (the graph gets sparser, so
    fewer draws collide), and the full-size fraction continues that trend
    below 1."""
    kept = []
    for scale in (12, 14, 16):
        rp, col = synth.rmat_csr(scale, 44, seed=synth.SEED_GRAPH)
        kept.append(col.shape[0] / ((1 << scale) * 44))
    full = STAND_INS[0][4] / ((1 << 25) * 44)
    assert np.all(np.diff(kept) > 0)
    assert kept[-1] < full < 1.0
