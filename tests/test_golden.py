"""The stored oracle values on an orbital subset of the headline workload
(tests/golden/make_subset_golden.py): the file regenerates its inputs, and
its numbers obey relations of Appendix B that the script did not use to
write them (the one-body term from the two-body term, the zero-body term
from the one-body term, the chemist symmetries of the unique entries)."""
import os

import numpy as np
import pytest

from paper_2304_07006_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "N128-occ16-Ng150k_subset.npz")


@pytest.fixture(scope="module")
def golden():
    g = np.load(GOLDEN, allow_pickle=False)
    return {k: g[k] for k in g.files}


def _full_block(g):
    """V2 on S^4 from its unique entries (a<=b, c<=d, pair(a,b)<=pair(c,d))."""
    nS = len(g["S"])
    V = np.full((nS,) * 4, np.nan)
    idx = g["idx"].astype(np.int64)
    for (a, b, c, d), v in zip(idx, g["V2u"]):
        for (p, q, r, s) in ((a, b, c, d), (b, a, c, d), (a, b, d, c), (b, a, d, c)):
            V[p, q, r, s] = v
            V[r, s, p, q] = v
    return V


def test_golden_regenerates_its_inputs(golden):
    p = inputs.make_workload("N128-occ16-Ng150k", lowdin=golden["X"])
    fp = inputs.input_fingerprint(p)
    assert np.all(np.abs(fp - golden["fingerprint"]) <= 1e-12 * np.abs(golden["fingerprint"]))
    # the stored orthonormalisation matrix orthonormalises the regenerated functions
    O = (p.phi * p.w) @ p.phi.T
    assert np.abs(O - np.eye(p.N)).max() < 1e-6
    S = golden["S"]
    assert len(S) == 24 and list(S[:16]) == list(range(16)) and len(set(S.tolist())) == 24


def test_golden_obeys_appendix_b_relations(golden):
    V = _full_block(golden)
    assert not np.isnan(V).any()
    nocc = 16
    k = np.arange(nocc)
    # Delta h_pq = -1/2 (2 sum_k V2[p,q,k,k] - sum_k V2[p,k,k,q]) on the subset
    h = -0.5 * (2.0 * np.einsum("pqkk->pq", V[:, :, k][:, :, :, k]) - np.einsum("pkkq->pq", V[:, k][:, :, k]))
    assert np.abs(h - golden["h1"]).max() < 1e-12 * max(1.0, np.abs(golden["h1"]).max())
    E0 = -(2.0 / 3.0) * np.trace(golden["h1"][:nocc, :nocc])
    assert abs(E0 - golden["E0"][0]) < 1e-12 * abs(E0)
    assert np.abs(golden["h1"] - golden["h1"].T).max() < 1e-12
