"""Throughput of the xTC folding on one MI355X.

One step = one whole pass of the hot path over the workload: prepare the
pair densities, then per grid chunk build K, form the intermediates and add
the two-body and one-/zero-body terms, finalising V2, h1 and E0 on the last
chunk.  Inputs are resident in HBM before the timed region starts.

The headline form is split-BF16 with three products (FP64 for the
occupied-occupied block and for the one-/zero-body reductions); the plain
FP64 path is run once beside it for the speedup and the max-abs error of
every output.

The value is algorithmic GFLOP/s:
    F_alg = 6 Ng^2 Npair + 8 Ng Npair^2 + (18 n + 10) Ng Npair
(K build, two-body assembly, intermediates; Npair = N(N+1)/2) divided by the
wall time of one step.  Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "xTC 2-body build GFLOP/s at N=128: FP64 vs split-BF16 at ≤1e-6 Eh error"
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "bf16x6": 2500.0}   # TFLOP/s, dense MFMA
TERMS = {"fp64": 1, "fp32": 1, "bf16x3": 3, "bf16x6": 6}                     # MFMA products per useful one
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3", "bf16x6": "bf16x6"}


def default_chunk(Ng, prec):
    """Equal-sized grid chunks, so every K-build launch covers the same rows."""
    parts = 10 if prec == "fp64" else 20
    return -(-Ng // parts)


def kernel_sources_hash():
    """Hash of the HIP sources the K build is made of (the traffic figures in
    profiles/ are only reported while it matches)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("xtc_device.h", "kernels_build_k.h", "kernels_lp.h", "kernels_prepare.h", "kernels_occ_i8.h",
              "occ_i8.hip", "xtc_api.hip"):
        with open(os.path.join(ROOT, "paper_2304_07006_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_record(prec, workload, chunk):
    """Per-launch HBM bytes of xtc_build_K from the committed counter summary."""
    path = os.path.join(ROOT, "profiles", "traffic_xtc_build_K.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    key = f"{workload}/{prec}/{chunk}"
    e = rec.get(key)
    if not e or e.get("sources") != kernel_sources_hash():
        return None
    return e


KBUILD_KERNELS = ("k_build_K_lp", "k_reduce_K", "k_build_K_occ_i8", "k_build_K_occ", "k_reduce_occ", "k_build_K_f64")


def traffic_from(fetch_dir, write_dir, workload, prec, chunk, path=None):
    """Write the per-launch HBM bytes of xtc_build_K into
    profiles/traffic_xtc_build_K.json from two counter runs of --probe
    (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE, --output-format csv).
    The 1 GiB copy of the probe calibrates both counters."""
    import csv
    import glob

    def per_kernel(d, counter):
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if len(files) != 1:
            raise SystemExit(f"expected one counter_collection.csv under {d}, found {len(files)}")
        disp = {}
        for row in csv.DictReader(open(files[0])):
            if row["Counter_Name"] != counter:
                continue
            k = (row["Dispatch_Id"], row["Kernel_Name"])
            disp[k] = disp.get(k, 0.0) + float(row["Counter_Value"])
        copy = [v for (_, n), v in disp.items() if "copy" in n.lower() and "fill" not in n.lower()]
        if len(copy) != 1:
            raise SystemExit(f"{counter}: expected one calibration copy dispatch, found {len(copy)}")
        factor = 2 ** 20 / copy[0]                   # counters are in KiB; the copy moves 2^30 bytes
        out = {}
        for (_, n), v in disp.items():
            short = n.split("(")[0].replace("void ", "").split("::")[-1].split("<")[0]
            if short in KBUILD_KERNELS:
                out[short] = out.get(short, 0.0) + v * 1024 * factor
        return out, factor

    fetch, ff = per_kernel(fetch_dir, "FETCH_SIZE")
    write, wf = per_kernel(write_dir, "WRITE_SIZE")
    path = path or os.path.join(ROOT, "profiles", "traffic_xtc_build_K.json")
    rec = json.load(open(path)) if os.path.exists(path) else {}
    rec[f"{workload}/{prec}/{chunk}"] = {
        "bytes_per_launch": sum(fetch.values()) + sum(write.values()),
        "sources": kernel_sources_hash(),
        "fetch_factor": ff, "write_factor": wf,
        "per_kernel_bytes": {k: {"fetch": fetch.get(k, 0.0), "write": write.get(k, 0.0)}
                             for k in sorted(set(fetch) | set(write))},
        "command": "rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) --output-format csv -d <dir> -o run "
                   "-- python -u bench.py --probe; python bench.py --traffic-from <fetch dir> <write dir>",
    }
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec[f"{workload}/{prec}/{chunk}"], indent=1))


def f_alg(N, n, Ng, nspin=1):
    """Algorithmic flops; the spin-resolved open-shell equations need the
    intermediates and the two-body contraction once per spin."""
    P = N * (N + 1) // 2
    return 6 * Ng * Ng * P + nspin * (8 * Ng * P * P + (18 * n + 10) * Ng * P)


def f_kbuild(N, rows, Ng):
    return 6 * rows * Ng * (N * (N + 1) // 2)


def apply_density(problem, spec):
    """Reference density of the workload: 'closed' (the closed-shell determinant
    of the workload), 'sa:ND,NS' (spin-averaged open shell, ND doubly and NS
    singly occupied orbitals), 'open:ND,NS' (the same determinant with the
    spin-resolved open-shell equations) or 'natural:NACT' (NACT natural
    orbitals with correlated occupation numbers).  Returns a short label."""
    import numpy as np
    from paper_2304_07006_amd import inputs
    if spec == "closed":
        return "closed-shell determinant"
    kind, _, arg = spec.partition(":")
    if kind == "sa":
        nd, ns = (int(x) for x in arg.split(","))
        problem.occ, problem.occ_n = inputs.sa_occupations(nd, ns)
        return f"spin-averaged open shell ({nd} doubly, {ns} singly occupied)"
    if kind == "open":
        nd, ns = (int(x) for x in arg.split(","))
        problem.occ, problem.occ_n, problem.occ_n_beta = inputs.open_shell_occupations(nd, ns)
        return f"open shell, spin-resolved ({nd} doubly, {ns} singly occupied)"
    if kind == "natural":
        nact = int(arg)
        problem.occ = np.arange(nact, dtype=np.int32)
        problem.occ_n = inputs.natural_occupations(nact, 2000)
        return f"{nact} natural orbitals with correlated occupations"
    raise SystemExit(f"unknown --density {spec}")


GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")


def load_golden(workload):
    """The oracle's outputs on an orbital subset of the workload (written by
    tests/golden/make_subset_golden.py), or None."""
    import numpy as np
    path = os.path.join(GOLDEN_DIR, f"{workload}_subset.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path, allow_pickle=False)
    return {k: g[k] for k in g.files}


def golden_inputs_match(problem, golden, rtol=1e-12):
    import numpy as np
    from paper_2304_07006_amd import inputs
    fp = inputs.input_fingerprint(problem)
    return bool(np.all(np.abs(fp - golden["fingerprint"]) <= rtol * np.abs(golden["fingerprint"])))


def golden_errors(golden, V2, h1, E0):
    """Max-abs error of device outputs against the stored oracle values on
    the subset S: V2 over its unique entries, h1 on S x S, E0."""
    import numpy as np
    import torch
    S = golden["S"].astype(np.int64)
    Sv = torch.as_tensor(S[golden["idx"].astype(np.int64)], device=V2.device)
    v = V2[Sv[:, 0], Sv[:, 1], Sv[:, 2], Sv[:, 3]].cpu().numpy()
    s = torch.as_tensor(S, device=h1.device)
    h = h1[s][:, s].cpu().numpy()
    return {"V2": float(np.abs(v - golden["V2u"]).max()), "h1": float(np.abs(h - golden["h1"]).max()),
            "E0": abs(float(E0.reshape(-1)[0].item()) - float(golden["E0"][0])),
            "orbitals": int(len(S))}


def short_kernel_name(name):
    """'void xtc::k_build_K_lp<0, 3, 3>(double const*, ...)' -> 'k_build_K_lp'."""
    return name.split("(")[0].replace("void ", "").split("::")[-1].split("<")[0].strip()


def profile_kernels(fn):
    """Device time per kernel (short name -> (launches, total seconds)) of
    the work fn() launches, from the torch profiler's device activity trace."""
    import torch
    from torch.profiler import ProfilerActivity, profile
    with profile(activities=[ProfilerActivity.CUDA]) as prof:
        fn()
        torch.cuda.synchronize()
    out = {}
    for ev in prof.events():
        if getattr(ev, "device_type", None) is None or str(ev.device_type) != "DeviceType.CUDA":
            continue
        k = short_kernel_name(ev.name)
        n, t = out.get(k, (0, 0.0))
        out[k] = (n + 1, t + ev.time_range.elapsed_us() * 1e-6)
    return out


I8_PEAK = 5000.0        # TOP/s, dense int8 MFMA
I8_PRODUCTS = 21        # digit products per useful one in the integer occupied block


def occ_i8_columns(nocc):
    """Pair columns the integer occupied block multiplies (16-pair tiles in
    groups of at most 9)."""
    nct = -(-(nocc * (nocc + 1) // 2) // 16)
    groups = -(-nct // 9)
    return 16 * groups * (-(-nct // groups))


def kernel_rooflines(times, N, nocc, Ng, prec):
    """Per-kernel algorithmic rate and fraction of the relevant peak for the
    contraction kernels of one step: the kernel's algorithmic flops per step
    (K build 6 Ng^2 Npair, occupied block 6 Ng^2 nOP, two-body GEMM
    8 Ng Npair^2) over its summed device time in that step.  The integer
    occupied block is rated by its executed int8 operations (21 digit
    products per useful one over its padded columns) against the int8 peak,
    and its useful rate is given beside it as an FP64-class rate."""
    P = N * (N + 1) // 2
    nOP = nocc * (nocc + 1) // 2
    table = {"k_build_K_lp": (6 * Ng * Ng * P, PEAK[prec]), "k_build_K_f64": (6 * Ng * Ng * P, PEAK["fp64"]),
             "k_build_K_occ": (6 * Ng * Ng * nOP, PEAK["fp64"]),
             "k_build_K_occ_i8": (6 * Ng * Ng * occ_i8_columns(nocc) * I8_PRODUCTS, I8_PEAK),
             "k_gemm_tn_lds": (8 * Ng * P * P, PEAK[prec]), "k_gemm_tn_lp": (8 * Ng * P * P, PEAK[prec]),
             "k_gemm2b_f64": (8 * Ng * P * P, PEAK["fp64"])}
    out = {}
    for k, (n, t) in sorted(times.items(), key=lambda kv: -kv[1][1]):
        e = {"launches": n, "avg_ms": t / n * 1e3, "total_ms": t * 1e3, "share_of_step": None}
        if k in table:
            f, peak = table[k]
            e.update(flop_per_step=f, tflops=f / t / 1e12, peak_tflops=peak, frac=f / t / 1e12 / peak)
        if k == "k_build_K_occ_i8":
            e.update(useful_flop_per_step=6 * Ng * Ng * nOP, useful_tflops=6 * Ng * Ng * nOP / t / 1e12)
        out[k] = e
    tot = sum(t for _, t in times.values())
    for k in out:
        out[k]["share_of_step"] = times[k][1] / tot
    return out


def run_gpu(problem, prec, steps, warmup, chunk, profile=False, kflags=0):
    import torch
    from paper_2304_07006_amd import xtc
    dp = xtc.device_problem(problem.xyz, problem.w, problem.phi, problem.occ,
                            occ_n=getattr(problem, "occ_n", None), occ_n_beta=getattr(problem, "occ_n_beta", None))
    ps = xtc.Pass(dp, xtc.PRECISIONS[prec], chunk)
    # the spin-resolved equations write three V2 blocks (aa, ab, bb) and two h1
    assert tuple(ps.V2.shape[:-4]) == ((3,) if dp.open_shell else ()), ps.V2.shape
    jas = xtc.make_jastrow(problem.jastrow)
    stream = torch.cuda.current_stream()
    kev = []

    def step(record):
        xtc.xtc_prepare(dp, ps.prec, ps.chunk, ps.ws)
        ch = ps.chunks()
        for i, (g0, g1) in enumerate(ch):
            flags = (xtc.XTC_RESET if i == 0 else 0) | (xtc.XTC_FINALIZE if i == len(ch) - 1 else 0)
            K = ps.K_view(g0, g1)
            if record:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            xtc.xtc_build_K(dp, jas, g0, g1, ps.prec | kflags, K, ps.ws)
            if record:
                e1.record(stream)
                kev.append((e0, e1, g1 - g0))
            xtc.xtc_contract_2body(dp, K, g0, g1, ps.prec, flags, ps.V2, ps.ws)
            xtc.xtc_contract_1body_0body(dp, K, g0, g1, ps.prec, flags | xtc.XTC_REUSE_INTERMEDIATES, ps.h1,
                                         ps.E0, ps.ws)

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    kt = [(a.elapsed_time(b) * 1e-3, rows) for a, b, rows in kev]
    times = None
    if profile:                       # one more step, untimed, under the profiler
        try:
            times = profile_kernels(lambda: step(False))
            busy = sum(t for _, t in times.values())
            if busy < 0.5 * dt:       # another profiler holds the device activity trace
                raise RuntimeError(f"kernel time {busy:.3f} s of a {dt:.3f} s step")
        except Exception as e:        # the breakdown is optional
            times = None
            print(f"[bench] kernel profile unavailable: {e}", file=sys.stderr, flush=True)
    return dict(sec=dt, kbuild=kt, outputs=(ps.V2, ps.h1, ps.E0), ws_bytes=ps.ws.numel(), kernel_times=times)


def probe(problem, prec, chunk):
    """Counter pass: a plain 1 GiB device-to-device copy (reads and writes
    exactly 2^30 bytes; it calibrates FETCH_SIZE / WRITE_SIZE) followed by one
    xtc_build_K launch of `chunk` rows (the dominant kernel)."""
    import torch
    from paper_2304_07006_amd import xtc
    a = torch.ones(2 ** 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    dp = xtc.device_problem(problem.xyz, problem.w, problem.phi, problem.occ)
    ps = xtc.Pass(dp, xtc.PRECISIONS[prec], chunk)
    xtc.xtc_prepare(dp, ps.prec, ps.chunk, ps.ws)
    xtc.xtc_build_K(dp, xtc.make_jastrow(problem.jastrow), 0, chunk, ps.prec, ps.K_view(0, chunk), ps.ws)
    torch.cuda.synchronize()
    print(f"[probe] copy 1 GiB + build_K {prec} rows=0..{chunk}", file=sys.stderr, flush=True)


def run_tc2(problem, prec, chunk, steps, warmup):
    """Two-body TC integrals pass (xtc_build_K + xtc_tc_2body over all chunks)."""
    import torch
    from paper_2304_07006_amd import inputs, xtc
    dphi = inputs.orbital_gradients(problem)
    xtc.tc_two_body(problem, dphi, prec, chunk)            # builds the library state once
    for _ in range(warmup):
        xtc.tc_two_body(problem, dphi, prec, chunk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        K2 = xtc.tc_two_body(problem, dphi, prec, chunk)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, K2


def f_backward(N, Ng, nspin=1):
    """Algorithmic flops of the adjoint as built: the K recompute and the Pi
    contraction (6 Ng^2 Npair each) and the seven X . Gbar products
    (2 Ng Npair^2 each) per spin channel."""
    P = N * (N + 1) // 2
    return 12 * Ng * Ng * P + nspin * 14 * Ng * P * P


def loss_weights_device(N, aux_seed, open_shell=False):
    """Seeded loss weights on the device: D symmetric [N][N] and G 8-fold
    symmetric [N]^4 (open shell: [2][N][N] and [3][N]^4, one per spin and
    per block aa, ab, bb)."""
    import torch
    nD, nG = (2, 3) if open_shell else (1, 1)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(aux_seed + 7)
    X = torch.randn((nD, N, N), generator=gen, device="cuda", dtype=torch.float64)
    D = 0.5 * (X + X.transpose(1, 2))
    G = torch.randn((nG, N, N, N, N), generator=gen, device="cuda", dtype=torch.float64)
    G = 0.25 * (G + G.permute(0, 2, 1, 3, 4) + G.permute(0, 1, 2, 4, 3) + G.permute(0, 2, 1, 4, 3))
    G = (0.5 * (G + G.permute(0, 3, 4, 1, 2))).contiguous()
    if nD == 1:
        D, G = D[0].contiguous(), G[0].contiguous()
    return D, G


def loss_value(V2, h1, E0, D, G):
    """E0 + <h1, D> + <V2, G> (device tensors), on the host."""
    return E0.reshape(-1)[0].item() + (h1 * D).sum().item() + (V2 * G).sum().item()


def run_backward(problem, prec, chunk, aux_seed, steps, warmup, keep=None):
    """Forward pass and adjoint (xtc_backward, K recomputed) of the loss
    L = E0 + <h1, D> + <V2, G>, D symmetric and G 8-fold symmetric, seeded on
    the device (open shell: one D per spin and one G per block aa, ab, bb).
    Returns seconds per forward and per backward, the gradient, and the Euler
    check |c . dL/dc - 2 L| / |2 L| (L is homogeneous of degree 2 in the
    power-Jastrow coefficients).  `keep`: a dict that receives host copies of
    the forward outputs and the loss."""
    import torch
    from paper_2304_07006_amd import xtc
    occ_n, occ_nb = getattr(problem, "occ_n", None), getattr(problem, "occ_n_beta", None)
    D, G = loss_weights_device(problem.N, aux_seed, occ_nb is not None)
    coef = [float(c) for c in problem.jastrow.coef]
    jas = xtc.power_jastrow(coef)
    dp = xtc.device_problem(problem.xyz, problem.w, problem.phi, problem.occ, occ_n=occ_n, occ_n_beta=occ_nb)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    # forward, then its workspace is released before the adjoint's is taken
    # (at N=160 each holds about half of the device memory)
    ps = xtc.Pass(dp, xtc.PRECISIONS[prec], chunk)
    tf = timed(lambda: ps.run(jas))
    L = loss_value(ps.V2, ps.h1, ps.E0, D, G)
    if keep is not None:              # host copies of the forward outputs
        keep.update(V2=ps.V2.cpu().numpy(), h1=ps.h1.cpu().numpy(), E0=float(ps.E0.cpu()[0]), L=L)
    del ps
    torch.cuda.empty_cache()
    pb = xtc.PRECISIONS[prec] | xtc.XTC_WITH_BACKWARD
    ws = torch.empty(xtc.xtc_workspace_size(dp, pb, chunk), dtype=torch.uint8, device="cuda")
    gc = torch.empty(len(coef), dtype=torch.float64, device="cuda")

    def bwd():
        xtc.xtc_prepare(dp, pb, chunk, ws)
        xtc.xtc_backward(dp, jas, pb, G, D, 1.0, gc, ws)

    tb = timed(bwd)
    g = gc.cpu().numpy()
    euler = abs(float(sum(c * x for c, x in zip(coef, g))) - 2 * L) / abs(2 * L)
    return tf, tb, g, euler, torch.cuda.max_memory_allocated()


def gemm_calibration(reps=10):
    """Executed rate of the vendor BF16 GEMM (torch.matmul -> hipBLASLt) on
    random normal operands: what a plain dense BF16 contraction sustains on
    this device, as a scale for the K build's executed MFMA rate."""
    import torch
    torch.manual_seed(0)
    rows = []
    for M, N, K in ((8192, 8192, 8192), (7520, 8704, 32768), (16384, 16384, 16384)):
        a = torch.randn(M, K, device="cuda", dtype=torch.bfloat16)
        b = torch.randn(K, N, device="cuda", dtype=torch.bfloat16)
        for _ in range(2):
            c = a @ b
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            c = a @ b
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        rows.append({"M": M, "N": N, "K": K, "ms": ms, "tflops": 2.0 * M * N * K / ms / 1e9})
        print(f"[calibration] bf16 GEMM {M}x{N}x{K}: {ms:.3f} ms, {rows[-1]['tflops']:.1f} TFLOP/s",
              file=sys.stderr, flush=True)
        del a, b, c
        torch.cuda.empty_cache()
    return rows


def host_info():
    """CPU model, cores this process may use and the BLAS threads numpy runs."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = None
    try:
        from threadpoolctl import threadpool_info
        blas = sum(int(i.get("num_threads", 0)) for i in threadpool_info() if i.get("user_api") == "blas") or None
    except Exception:
        pass
    return {"cpu_model": model, "cores": len(os.sched_getaffinity(0)), "blas_threads": blas}


def cpu_baseline(name, budget_rows, nvirt=8):
    """The oracle (Appendix-B equations, numpy FP64) on the workload's orbital
    subset occ + `nvirt` virtual orbitals (exact for that subset) on a
    `budget_rows`-point grid of the same generator, where, as in the whole
    workload, the K build dominates the work.  Its rate (algorithmic flops of
    the subset problem over the wall time) is extrapolated to the whole
    workload, labelled as such."""
    import numpy as np
    from paper_2304_07006_amd import inputs
    from oracle import factorised
    wl = inputs.WORKLOADS[name]
    p = inputs.make_workload(name, Ng=budget_rows)
    occ = [int(k) for k in p.occ]
    rest = np.array([k for k in range(p.N) if k not in set(occ)])
    virt = np.sort(np.random.default_rng(7).choice(rest, nvirt, replace=False))
    S = np.array(occ + [int(k) for k in virt])
    t0 = time.perf_counter()
    factorised.closed_shell(p.xyz, p.w, p.phi[S], np.arange(len(occ)), p.jastrow)
    dt = time.perf_counter() - t0
    F = f_alg(len(S), wl.nocc, budget_rows)
    info = host_info()
    rate = F / dt
    return {"value": rate / 1e9, "unit": "GFLOP/s", "cores": info["cores"], "kind": "oracle",
            "sample": f"Appendix-B oracle (numpy FP64) on orbitals occ+{nvirt} virtual ({len(S)} of {wl.N}; "
                      f"exact for that subset) of {name}'s generator on a {budget_rows}-point grid; "
                      f"{dt:.1f} s wall; rate = F_alg(N={len(S)}, n={wl.nocc}, Ng={budget_rows}) / time",
            "seconds": dt, "cpu_model": info["cpu_model"], "blas_threads": info["blas_threads"],
            "oracle_threads": min(16, info["cores"]),
            "k_build_share_of_sample_flops": f_kbuild(len(S), budget_rows, budget_rows) / F,
            # the whole workload's F_alg at the sample's rate (extrapolated, not run)
            "full_workload_seconds_extrapolated": f_alg(wl.N, wl.nocc, wl.Ng) / rate}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="N128-occ16-Ng150k")
    ap.add_argument("--prec", default="bf16x3", choices=list(PEAK))
    ap.add_argument("--compare", default="fp64,fp32",
                    help="comma-separated forms run once beside the headline one, the first being the reference "
                         "the others are compared against ('none' to skip; the TC integrals use the first)")
    ap.add_argument("--chunk", type=int, default=None,
                    help="grid rows per chunk (default: Ng/10 for FP64, Ng/20 for the reduced forms: equal launches)")
    ap.add_argument("--cpu-rows", type=int, default=30000,
                    help="grid points of the CPU oracle sample (orbital subset), 10-30 s on the host (0: skip)")
    ap.add_argument("--density", default="closed",
                    help="reference density: closed | sa:ND,NS | open:ND,NS | natural:NACT (see apply_density)")
    ap.add_argument("--tc2", action="store_true",
                    help="time the two-body TC integrals (K build + xtc_tc_2body) instead of the xTC folding")
    ap.add_argument("--backward", action="store_true",
                    help="time forward + adjoint (xtc_backward) on a power-Jastrow workload "
                         "(default workload then N96-occ12-Ng100k)")
    ap.add_argument("--occ-fp64", action="store_true",
                    help="compute the reduced forms' occupied-occupied block of K with FP64 MFMA "
                         "(XTC_K_OCC_FP64) instead of the integer-sliced products")
    ap.add_argument("--probe", action="store_true",
                    help="counter pass: one 1 GiB device copy (calibration) and one K-build launch, no JSON")
    ap.add_argument("--gemm-calibration", action="store_true",
                    help="time the vendor BF16 GEMM (torch.matmul) on random data instead, one JSON line")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two --probe counter runs into profiles/traffic_xtc_build_K.json (no GPU)")
    args = ap.parse_args()
    if args.traffic_from:
        from paper_2304_07006_amd import inputs
        wl = inputs.WORKLOADS[args.workload]
        traffic_from(*args.traffic_from, args.workload, args.prec, args.chunk or default_chunk(wl.Ng, args.prec))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the grid-row sharding is described in the design notes). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2304_07006_amd import inputs, xtc
    xtc.load()
    if not torch.cuda.is_available():
        print("no HIP device", file=sys.stderr)
        sys.exit(1)
    if args.gemm_calibration:
        print(json.dumps({"calibration": "vendor BF16 GEMM (torch.matmul, random normal operands)",
                          "runs": gemm_calibration()}), flush=True)
        return
    if args.backward and args.workload == ap.get_default("workload"):
        args.workload = "N96-occ12-Ng100k"
    wl = inputs.WORKLOADS[args.workload]
    golden = load_golden(args.workload) if args.density == "closed" else None
    problem = inputs.make_workload(args.workload, lowdin=golden["X"] if golden else None)
    if golden and not golden_inputs_match(problem, golden):
        print("[bench] regenerated inputs differ from the stored oracle values' inputs: no oracle errors",
              file=sys.stderr, flush=True)
        golden = None
    density = apply_density(problem, args.density)
    nref = len(problem.occ)
    chunk = args.chunk or default_chunk(wl.Ng, args.prec)
    if args.probe:
        probe(problem, args.prec, chunk)
        return
    if args.backward:
        if wl.jastrow_kind == "pade":
            print("the adjoint needs a power-Jastrow workload", file=sys.stderr)
            sys.exit(2)
        nspin = 2 if getattr(problem, "occ_n_beta", None) is not None else 1
        Ff, Fb = f_alg(wl.N, nref, wl.Ng, nspin), f_backward(wl.N, wl.Ng, nspin)
        print(f"[bench] backward {args.workload} prec={args.prec} chunk={chunk}", file=sys.stderr, flush=True)
        tf, tb, g, euler, peak_mem = run_backward(problem, args.prec, chunk, wl.aux_seed, args.steps, args.warmup)
        line = {"metric": "xTC forward + adjoint GFLOP/s (loss E0 + <h1,D> + <V2,G>, gradient in the Jastrow coefficients)",
                "value": (Ff + Fb) / (tf + tb) / 1e9, "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
                "warmup": args.warmup, "ms_per_step": (tf + tb) * 1e3, "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": DTYPE[args.prec], "data": "synthetic",
                "config": {"workload": args.workload, "N": wl.N, "nocc": nref, "Ng": wl.Ng, "prec": args.prec,
                           "chunk_rows": chunk, "density": density, "F_fwd": Ff, "F_bwd": Fb},
                "forward_s": tf, "backward_s": tb, "forward_tflops": Ff / tf / 1e12,
                "backward_tflops": Fb / tb / 1e12, "euler_rel": euler, "peak_device_bytes": peak_mem,
                "grad_head": [float(x) for x in g[:4]]}
        print(json.dumps(line), flush=True)
        return
    if args.tc2:
        P = wl.N * (wl.N + 1) // 2
        Ftc = 6 * wl.Ng ** 2 * P + 2 * wl.Ng ** 2 * P + 2 * wl.Ng * P * P + 6 * wl.Ng * wl.N ** 2 * P
        sec, K2 = run_tc2(problem, args.prec, chunk, args.steps, args.warmup)
        line = {"metric": "two-body TC integrals GFLOP/s (K build + F = S rho + A, B contractions)",
                "value": Ftc / sec / 1e9, "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
                "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": DTYPE[args.prec] + "+f64", "data": "synthetic",
                "config": {"workload": args.workload, "N": wl.N, "Ng": wl.Ng, "prec": args.prec,
                           "chunk_rows": chunk, "F_flop": Ftc}}
        tc_ref = args.compare.split(",")[0]
        if tc_ref not in ("", "none", args.prec):
            sec_c, K2c = run_tc2(problem, tc_ref, default_chunk(wl.Ng, tc_ref), 1, 0)
            line["forms"] = {tc_ref: {"s_per_step": sec_c,
                                            "max_abs_err": (K2 - K2c).abs().max().item(),
                                            "max_abs": K2c.abs().max().item()}}
        print(json.dumps(line), flush=True)
        return
    print(f"[bench] {args.workload} prec={args.prec} chunk={chunk} warmup={args.warmup} steps={args.steps}",
          file=sys.stderr, flush=True)
    from paper_2304_07006_amd import xtc
    kflags = xtc.XTC_K_OCC_FP64 if args.occ_fp64 else 0
    r = run_gpu(problem, args.prec, args.steps, args.warmup, chunk, profile=True, kflags=kflags)
    nspin = 2 if getattr(problem, "occ_n_beta", None) is not None else 1
    F = f_alg(wl.N, nref, wl.Ng, nspin)
    def form_rates(sec):
        # whole-step algorithmic rate, also as a fraction of the FP64 and FP32 MFMA peaks
        tf = F / sec / 1e12
        return {"s_per_step": sec, "gflops": tf * 1e3, "frac_of_fp64_peak": tf / PEAK["fp64"],
                "frac_of_fp32_peak": tf / PEAK["fp32"]}

    forms = {args.prec: form_rates(r["sec"])}
    if golden:
        forms[args.prec]["max_abs_err_vs_oracle"] = golden_errors(golden, *r["outputs"])
        print(f"[bench] {args.prec} vs oracle subset: {forms[args.prec]['max_abs_err_vs_oracle']}",
              file=sys.stderr, flush=True)
    # comparison forms, one step each: the first (FP64 by default) is the
    # reference the headline form and every later one are compared against
    cmp = [c for c in args.compare.split(",") if c and c not in ("none", args.prec)]
    if cmp:
        def errors(x, y):
            return {"V2": (x[0] - y[0]).abs().max().item(), "h1": (x[1] - y[1]).abs().max().item(),
                    "E0": (x[2] - y[2]).abs().max().item()}

        head = tuple(t.clone() for t in r["outputs"])
        del r["outputs"]
        torch.cuda.empty_cache()
        ref = ref_sec = ref_name = None
        for form in cmp:
            print(f"[bench] comparison form {form}: one step", file=sys.stderr, flush=True)
            rc = run_gpu(problem, form, 1, 0, default_chunk(wl.Ng, form), profile=form == "fp64", kflags=kflags)
            if rc.get("kernel_times"):
                forms[form + "_kernels"] = kernel_rooflines(rc["kernel_times"], wl.N, nref, wl.Ng, form)
            outs = rc.pop("outputs")
            forms[form] = form_rates(rc["sec"])
            if golden:
                forms[form]["max_abs_err_vs_oracle"] = golden_errors(golden, *outs)
            if ref is None:
                ref, ref_sec, ref_name = outs, rc["sec"], form
                err = errors(head, ref)
                forms[args.prec]["max_abs_err_vs_" + form] = err
                forms[args.prec]["speedup_vs_" + form] = rc["sec"] / r["sec"]
            else:
                err = errors(outs, ref)
                forms[form]["max_abs_err_vs_" + ref_name] = err
                forms[form]["speedup_vs_" + ref_name] = ref_sec / rc["sec"]
                del outs
            print(f"[bench] {form}: {rc['sec']:.3f} s/step; max|err| {err}", file=sys.stderr, flush=True)
            del rc
            torch.cuda.empty_cache()
        del head, ref
        torch.cuda.empty_cache()
    # roofline of the dominant kernel (K build): algorithmic flops per launch over
    # its average launch duration from HIP events on the launch stream
    tot_f = sum(f_kbuild(wl.N, rows, wl.Ng) for _, rows in r["kbuild"])
    tot_t = sum(t for t, _ in r["kbuild"])
    nl = len(r["kbuild"])
    achieved = (tot_f / nl) / (tot_t / nl) / 1e12
    peak = PEAK[args.prec]
    print(f"[bench] step {r['sec']:.3f} s; K build {nl} launches, avg {tot_t / nl * 1e3:.1f} ms, "
          f"{achieved:.1f} TFLOP/s", file=sys.stderr, flush=True)
    cpu = None
    if args.cpu_rows > 0 and args.density == "closed":
        print(f"[bench] CPU oracle sample: {args.cpu_rows} grid points", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.workload, args.cpu_rows)
    out = {
        "metric": METRIC,
        "value": F / r["sec"] / 1e9,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["sec"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.prec],
        "data": "synthetic",
        "config": {"workload": args.workload, "N": wl.N, "nocc": nref, "Ng": wl.Ng, "prec": args.prec,
                   "chunk_rows": chunk, "jastrow": wl.jastrow_kind, "density": density, "F_alg_flop": F,
                   "workspace_bytes": r["ws_bytes"], "occupied_block": "fp64" if args.occ_fp64 else "int8-sliced"},
        "roofline": {"bound": "mfma", "kernel": "xtc_build_K", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": (tr["bytes_per_launch"] if (tr := traffic_record(args.prec, args.workload, chunk))
                                 else None),
                     "per_launch_flop": tot_f / nl, "avg_launch_ms": tot_t / nl * 1e3,
                     "executed_mfma_frac": achieved * TERMS[args.prec] / peak},
        "forms": forms,
        "kernels": (kernel_rooflines(r["kernel_times"], wl.N, nref, wl.Ng, args.prec)
                    if r.get("kernel_times") else None),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
