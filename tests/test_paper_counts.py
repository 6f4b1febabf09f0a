"""Golden pin of the edge-count reading against the paper's printed tables.

With the new edge eigenproblem an edge shared by |n(E)| subdomains with
|N_E| selected eigenvectors contributes r_E = min(n_E, (|n(E)| - 1) |N_E|)
primal unknowns (the generic rank of the SVD step).  On the paper's 2x2x2
partitions (6 edges, |n(E)| = 4, n_E = m - 1) every printed ABDDC-NEW pnumE
must therefore be a sum of at most 6 values from {min(3 j, m - 1)}, while the
old method (one primal unknown per eigenvector) is not so restricted.  The
face stage is shared by both methods, so pnumF must agree row by row."""
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def _representable(total, m, nedges=6):
    vals = sorted({min(3 * j, m - 1) for j in range(0, m)})
    reach = {0}
    for _ in range(nedges):
        reach = reach | {a + v for a in reach for v in vals}
    return total in reach


def test_new_edge_counts_fit_rank_rule():
    data = json.load(open(os.path.join(HERE, "golden", "paper_primal_counts.json")))
    old_misfit = 0
    for row in data["tables"]:
        m = row["m"]
        for (fo, eo), (fn, en) in zip(row["old"], row["new"]):
            assert fo == fn, row
            assert _representable(en, m), (row, en)
            old_misfit += not _representable(eo, m)
    assert old_misfit > 0
