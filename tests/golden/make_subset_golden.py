"""Write the oracle's outputs on an orbital subset of a full-size workload.

    python tests/golden/make_subset_golden.py [--workload N128-occ16-Ng150k]
                                              [--virtuals 8] [--seed 7]

The workload's inputs come from the seeded generator; its orthonormalisation
matrix X = S^{-1/2} is computed here once and stored with the results, so that
any host regenerates the same orbitals phi = X chi to about 1e-13 (computing
S^{-1/2} again on another host moves phi by about cond(S) x 1e-16, 4e-10 at
N=128, which moves E0 by up to 4e-9 Eh).  The orbitals S = occ + `virtuals`
seeded virtual ones are passed to the Appendix-B oracle (oracle.factorised):
the two-body term restricted to S, the one-body term restricted to S and the
zero-body term are exact there, because every sum over the reference density
runs over occupied orbitals only (pinned in tests/test_oracle.py).  Only the
oracle and the input generator are called.

Stored (numpy .npz, no pickles): S, X, the input fingerprint
(inputs.input_fingerprint), the unique two-body entries V2[S[a], S[b], S[c],
S[d]] with a <= b, c <= d and pair(a, b) <= pair(c, d) (indices in idx), h1 on
S x S and E0.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_2304_07006_amd import inputs  # noqa: E402
from oracle import factorised  # noqa: E402


def golden_path(workload: str) -> str:
    return os.path.join(HERE, f"{workload}_subset.npz")


def subset_orbitals(p, n_virtual: int, seed: int) -> np.ndarray:
    occ = [int(k) for k in p.occ]
    rest = np.array([k for k in range(p.N) if k not in set(occ)])
    virt = np.sort(np.random.default_rng(seed).choice(rest, n_virtual, replace=False))
    return np.array(occ + [int(k) for k in virt], dtype=np.int64)


def unique_index(nS: int) -> np.ndarray:
    """[M][4] local indices (a, b, c, d): a <= b, c <= d, pair(a, b) <= pair(c, d)."""
    pairs = [(a, b) for a in range(nS) for b in range(a, nS)]
    return np.array([(*pairs[i], *pairs[j]) for i in range(len(pairs)) for j in range(i, len(pairs))],
                    dtype=np.uint8 if nS < 256 else np.int32)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="N128-occ16-Ng150k")
    ap.add_argument("--virtuals", type=int, default=8)
    ap.add_argument("--seed", type=int, default=7)
    args = ap.parse_args()
    t0 = time.time()
    wl = inputs.WORKLOADS[args.workload]
    p0 = inputs.make_workload(args.workload)
    X = inputs.lowdin_matrix(p0.chi, p0.w)
    p = inputs.make_workload(args.workload, lowdin=X)
    S = subset_orbitals(p, args.virtuals, args.seed)
    nocc = len(p.occ)
    print(f"[golden] {args.workload}: subset of {len(S)} orbitals, Ng={p.Ng}", flush=True)
    V2, h1, E0 = factorised.closed_shell(p.xyz, p.w, p.phi[S], np.arange(nocc), p.jastrow)
    idx = unique_index(len(S))
    V2u = V2[idx[:, 0], idx[:, 1], idx[:, 2], idx[:, 3]]
    meta = {"workload": args.workload, "N": wl.N, "nocc": wl.nocc, "Ng": wl.Ng, "virtuals": args.virtuals,
            "seed": args.seed, "oracle": "oracle.factorised.closed_shell on the orbital subset",
            "command": f"python tests/golden/make_subset_golden.py --workload {args.workload} "
                       f"--virtuals {args.virtuals} --seed {args.seed}",
            "seconds": round(time.time() - t0, 1)}
    np.savez_compressed(golden_path(args.workload), S=S, X=X, fingerprint=inputs.input_fingerprint(p),
                        idx=idx, V2u=V2u, h1=h1, E0=np.array([E0]), meta=np.array(json.dumps(meta)))
    print(f"[golden] E0 = {E0:.12f}, max|V2| {np.abs(V2).max():.3e}; {meta['seconds']} s -> "
          f"{golden_path(args.workload)}", flush=True)


if __name__ == "__main__":
    main()
