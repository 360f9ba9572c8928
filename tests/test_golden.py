"""The stored oracle values on orbital subsets of the measured workloads
(tests/golden/make_subset_golden.py): each file regenerates its inputs, and
its numbers obey relations of Appendix B that the script did not use to
write them (the one-body term from the two-body term, the zero-body term
from the one-body term, the chemist symmetries of the unique entries)."""
import json
import os

import numpy as np
import pytest

from paper_2304_07006_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
STORED = ["N128-occ16-Ng150k", "N96-occ12-Ng100k", "N160-occ20-Ng250k"]


def _load(name):
    path = os.path.join(HERE, "golden", f"{name}_subset.npz")
    if not os.path.exists(path):
        pytest.fail(f"{path} is missing")
    g = np.load(path, allow_pickle=False)
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


@pytest.mark.parametrize("name", STORED)
def test_stored_values_regenerate_their_inputs(name):
    g = _load(name)
    meta = json.loads(str(g["meta"]))
    wl = inputs.WORKLOADS[name]
    assert meta["workload"] == name and meta["N"] == wl.N and meta["Ng"] == wl.Ng
    p = inputs.make_workload(name, lowdin=g["X"])
    fp = inputs.input_fingerprint(p)
    assert np.all(np.abs(fp - g["fingerprint"]) <= 1e-12 * np.abs(g["fingerprint"]))
    # the stored orthonormalisation matrix orthonormalises the regenerated functions
    O = (p.phi * p.w) @ p.phi.T
    assert np.abs(O - np.eye(p.N)).max() < 1e-6
    S = g["S"]
    assert len(S) == wl.nocc + meta["virtuals"] and list(S[:wl.nocc]) == list(range(wl.nocc))
    assert len(set(S.tolist())) == len(S)


@pytest.mark.parametrize("name", STORED)
def test_stored_values_obey_appendix_b_relations(name):
    g = _load(name)
    V = _full_block(g)
    assert not np.isnan(V).any()
    nocc = inputs.WORKLOADS[name].nocc
    k = np.arange(nocc)
    # Delta h_pq = -1/2 (2 sum_k V2[p,q,k,k] - sum_k V2[p,k,k,q]) on the subset
    h = -0.5 * (2.0 * np.einsum("pqkk->pq", V[:, :, k][:, :, :, k]) - np.einsum("pkkq->pq", V[:, k][:, :, k]))
    assert np.abs(h - g["h1"]).max() < 1e-12 * max(1.0, np.abs(g["h1"]).max())
    E0 = -(2.0 / 3.0) * np.trace(g["h1"][:nocc, :nocc])
    assert abs(E0 - g["E0"][0]) < 1e-12 * abs(E0)
    assert np.abs(g["h1"] - g["h1"].T).max() < 1e-12
