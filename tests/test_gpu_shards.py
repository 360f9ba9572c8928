"""The grid-row sharding that a multi-GPU run would use, emulated on one GPU:
every shard owns a contiguous range of output rows g (the sums over g' still
run over the whole grid), accumulates and finalizes its own partial outputs,
and the shard outputs are summed in a fixed order.  V2, h1 and E0 are linear
in the per-row accumulators, so the sum must equal the unsharded pass; with
shard boundaries on the unsharded chunk boundaries every chunk's arithmetic
is the same, and only the FP64 order of the cross-chunk sums differs."""
import numpy as np
import pytest

from paper_2304_07006_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _rows_pass(xtc, dp, jas, prec, chunk, r0, r1):
    """One workspace, chunks of `chunk` rows over output rows [r0, r1)."""
    import torch
    ps = xtc.Pass(dp, prec, chunk)
    xtc.xtc_prepare(dp, ps.prec, ps.chunk, ps.ws)
    ch = [(g0, min(r1, g0 + chunk)) for g0 in range(r0, r1, chunk)]
    for i, (g0, g1) in enumerate(ch):
        flags = (xtc.XTC_RESET if i == 0 else 0) | (xtc.XTC_FINALIZE if i == len(ch) - 1 else 0)
        K = ps.K_view(g0, g1)
        xtc.xtc_build_K(dp, jas, g0, g1, ps.prec, K, ps.ws)
        xtc.xtc_contract_2body(dp, K, g0, g1, ps.prec, flags, ps.V2, ps.ws)
        xtc.xtc_contract_1body_0body(dp, K, g0, g1, ps.prec, flags | xtc.XTC_REUSE_INTERMEDIATES, ps.h1, ps.E0,
                                     ps.ws)
    torch.cuda.synchronize()
    return ps.V2.cpu().numpy(), ps.h1.cpu().numpy(), float(ps.E0.cpu()[0])


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_row_shards_sum_to_the_whole(torch_cuda, prec):
    from paper_2304_07006_amd import xtc
    p = inputs.make_problem(24, 4, 1900, 6, "chain", "pade", seed=81)
    chunk, bounds = 352, [0, 704, 1408, 1900]          # three shards on chunk boundaries, ragged last
    print(f"case: N24 Ng1900 {prec} shards {bounds} chunk {chunk}", flush=True)
    dp = xtc.device_problem(p.xyz, p.w, p.phi, p.occ)
    jas = xtc.make_jastrow(p.jastrow)
    P = xtc.PRECISIONS[prec]
    V2, h1, E0 = _rows_pass(xtc, dp, jas, P, chunk, 0, p.Ng)
    parts = [_rows_pass(xtc, dp, jas, P, chunk, a, b) for a, b in zip(bounds[:-1], bounds[1:])]
    V2s = parts[0][0] + parts[1][0] + parts[2][0]
    h1s = parts[0][1] + parts[1][1] + parts[2][1]
    E0s = parts[0][2] + parts[1][2] + parts[2][2]
    scale = max(1.0, float(np.abs(V2).max()), abs(E0))
    eV, eh, eE = np.abs(V2s - V2).max(), np.abs(h1s - h1).max(), abs(E0s - E0)
    print(f"  |dV2| {eV:.2e} |dh1| {eh:.2e} |dE0| {eE:.2e}; shard E0 {[round(x[2], 6) for x in parts]}", flush=True)
    assert eV < 1e-13 * scale and eh < 1e-13 * scale and eE < 1e-13 * scale
    assert all(np.abs(x[0]).max() > 0 for x in parts)        # every shard contributes
