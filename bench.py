"""Benchmark of the hot path: blocks + Wick-term sum for every time slice.

One step = the baryon blocks of every kind on every time slice of every
configuration (HIP, MFMA) followed by the FP64 sum over the deduplicated term
table for every (configuration, time slice), i.e. one full C(t) set. Inputs are
seeded synthetic propagators, already resident in HBM when the timed region
starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--precision p64]

Workloads: 2H-4^3x8 (small case), 3He-16^3x32 (default), 4He-24^3x48,
7Li-32^3x64 (the 4He and 3H cluster correlators, batched), batch64-16^3x32
(64 complex64 configurations: 8 2H, 24 3He, 32 4He correlators in one
graph-captured batch). Prints one JSON line. Only the ``cpu_baseline`` leg
uses the oracle.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Wick terms/s + block TFLOP/s per C(t) set, FP64 vs split-FP32 at 1e-8 rel"

# name -> dims (X, Y, Z, T), n_cfg, storage, seed workload id, items [(nucleus, cfg)], default precision
WORKLOADS = {
    "2H-4^3x8": ((4, 4, 4, 8), 1, "c128", 1, [("2H", 0)], "p64"),
    "3He-16^3x32": ((16, 16, 16, 32), 1, "c128", 2, [("3He", 0)], "p64"),
    "4He-24^3x48": ((24, 24, 24, 48), 1, "c128", 3, [("4He", 0)], "p64"),
    "7Li-32^3x64": ((32, 32, 32, 64), 1, "c128", 4, [("4He", 0), ("3H", 0)], "p32"),
    "batch64-16^3x32": ((16, 16, 16, 32), 64, "c64", 5,
                        [("2H", c) for c in range(8)] + [("3He", c) for c in range(8, 32)]
                        + [("4He", c) for c in range(32, 64)], "p64"),
}
DEFAULT = "3He-16^3x32"

# point-sink workloads (determinant method): name -> nucleus, dims, seed workload id
POINT_WORKLOADS = {
    "point-2H-24^3x8": ("2H", (24, 24, 24, 8), 11),
    "point-3He-24^3x8": ("3He", (24, 24, 24, 8), 12),
    "point-4He-24^3x8": ("4He", (24, 24, 24, 8), 13),
}
# correlation-matrix workloads (GEVP): name -> basis, dims, seed workload id
GEVP_WORKLOADS = {
    "gevp-2H-16^3x32": ("2H: n^T C g5 P+ p, n^T C g5 P- p, n^T C g5 p", (16, 16, 16, 32), 21),
}

# the paper's point-sink times per time slice at 24^3, seconds (context, other hardware):
# determinant method B on one i7-12th-gen core (method comparison table of Sec. 3.3)
# and its CUDA code (timing tables of Sec. 4)
PAPER_POINT_24 = {"2H": {"method_B_1core": 34.15, "cuda_V100": 0.34, "cuda_A100": 0.15},
                  "3He": {"method_B_1core": 2754.16, "cuda_V100": 5.24},
                  "4He": {"method_B_1core": 3246.38, "cuda_V100": 24.72}}


def laplace_cmacs(n):
    """Complex multiply-adds of all minors of one row set: sum_k binom(12, k) k."""
    from math import comb
    return sum(comb(12, k) * k for k in range(1, n + 1))

PEAK_TFLOPS = {"p64": 78.6, "p32": 157.3, "pb3": 2500.0, "pb6": 2500.0}
PEAK_NAME = {"p64": "FP64 MFMA", "p32": "FP32 MFMA", "pb3": "BF16 MFMA", "pb6": "BF16 MFMA"}

# algorithmic flops per site of the nucleon-form block build: block kinds per
# nucleus, and the distinct E-row sets (nonzero diquark-matrix entries of each;
# a p group and its n twin with an antisymmetric diquark matrix share one)
KINDS = {"2H": 4, "3He": 9, "3H": 9, "4He": 4}
EROWS = {"2H": [4], "3He": [2, 2], "3H": [2, 2], "4He": [4]}


def block_flops_per_site(nucleus):
    """GEMM: 12 rows (i1) per kind x 144 columns x 3 E rows x 8 flops per complex
    multiply-add; E rows: per nonzero diquark entry 6 complex products and
    adds for the three colour cross products (8 flops each) per column."""
    gemm = 12 * KINDS[nucleus] * 144 * 3 * 8
    erow = sum(144 * npair * 6 * 8 for npair in EROWS[nucleus])
    return gemm + erow


def kernel_source_hash():
    h = hashlib.sha256()
    # the kernels, and the host code that picks table forms and launch shapes
    for f in ("kernels.hip", "kernels.hpp", "api.hip"):
        h.update(open(os.path.join(ROOT, "paper_2411_08962_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def note(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def gen_inputs(wid, n_cfg, dims, dtype):
    import wick_inputs as wi
    hu = np.empty((n_cfg, dims[3], dims[2], dims[1], dims[0], 12, 12), dtype=dtype)
    hd = np.empty_like(hu)
    for c in range(n_cfg):
        hu[c] = wi.propagator(wid, c, 0, dims, dtype)
        hd[c] = wi.propagator(wid, c, 1, dims, dtype)
    return hu, hd


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 20; 3 for point-sink workloads)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT,
                    choices=sorted(WORKLOADS) + sorted(POINT_WORKLOADS) + sorted(GEVP_WORKLOADS))
    ap.add_argument("--precision", default=None, help="p64, p32, pb3, pb6 (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-split", action="store_true", help="skip the split-precision comparison")
    ap.add_argument("--no-truncation", action="store_true", help="skip the important-term truncation figures")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the default launch shapes instead of tuning them before the timed region")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device copy 5 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1 "
              "(multi-GPU sharding is a design note, not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        import torch
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read_per_launch": a.numel() * 8,
                          "bytes_written_per_launch": a.numel() * 8, "launches": 5}))
        return

    if args.steps is None:
        args.steps = 3 if args.workload in POINT_WORKLOADS else 20
    if args.workload in POINT_WORKLOADS:
        return point_bench(args)
    if args.workload in GEVP_WORKLOADS:
        return gevp_bench(args)

    import torch
    import paper_2411_08962_amd as W

    dims, n_cfg, dts, wid, items, prec0 = WORKLOADS[args.workload]
    prec = args.precision or prec0
    X, Y, Z, T = dims
    V = X * Y * Z
    dtype = np.complex128 if dts == "c128" else np.complex64
    t0 = time.time()
    hu, hd = gen_inputs(wid, n_cfg, dims, dtype)
    du, dd = torch.from_numpy(hu).cuda(), torch.from_numpy(hd).cuda()
    t_gen = time.time() - t0
    nuclei = sorted({n for n, _ in items}, key=lambda n: [m for m, _ in items].index(n))
    t0 = time.time()
    plans = {n: W.plan_std(n, 0) for n in nuclei}
    t_plan = time.time() - t0
    note(f"inputs {t_gen:.1f} s, plans {t_plan:.1f} s")
    t_tune = 0.0
    if not args.no_autotune:
        # launch shapes tuned on scratch inputs of this lattice (outside the timed region)
        t0 = time.time()
        for n in nuclei:
            for p in ([prec] if len(items) > 1 or args.no_split else [prec, "p32", "pb3", "pb6"]):
                W.autotune(plans[n], dims, dts, p)
        t_tune = time.time() - t0
        note(f"autotune {t_tune:.1f} s")
    single = len(items) == 1
    if single:
        pl = plans[nuclei[0]]
        A, K, N = pl.info()
        B = torch.empty((n_cfg, T, K, W.BLOCK_LEN, 2), dtype=torch.float64, device="cuda")
        C = torch.empty((n_cfg, T, 2), dtype=torch.float64, device="cuda")

        def step(p=prec):
            W.blocks(pl, du, dd, p, out=B)
            W.contract(pl, B, out=C)
    else:
        plist = [plans[n] for n in nuclei]
        bitems = [(nuclei.index(n), c) for n, c in items]
        C = torch.empty((len(items), T, 2), dtype=torch.float64, device="cuda")

        def step(p=prec, graph=True):
            W.correlator(plist, bitems, du, dd, p, use_graph=graph, out=C)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    W.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    W.profile(False)
    kernels = ("blocks", "blocks_reduce", "contract", "contract_finalize")
    prof = {k: W.profile_read(k) for k in kernels}
    graph_ms = None
    if not single:
        # kernel events cannot sit inside the captured graph: the per-kernel
        # durations come from the same batch launched eagerly
        graph_ms = W.profile_read("correlator")
        step(graph=False)
        torch.cuda.synchronize()
        W.profile(True)
        for _ in range(args.steps):
            step(graph=False)
        torch.cuda.synchronize()
        W.profile(False)
        prof = {k: W.profile_read(k) for k in kernels}
        eager = W.profile_read("correlator")
        graph_ms = {"graph_launch_ms": graph_ms[1] / max(graph_ms[0], 1),
                    "eager_batch_ms": eager[1] / max(eager[0], 1)}

    note(f"timed {args.steps} steps: {1e3 * dt / args.steps:.3f} ms/step")
    step_s = dt / args.steps
    n_term_evals = sum(plans[n].n_terms * T for n, _ in items)
    flops_launch = sum(block_flops_per_site(n) * V * T for n, _ in items)
    gemm_equiv = sum(165888.0 * plans[n].n_kinds * V * T for n, _ in items)
    nb, ms_b = prof["blocks"]
    avg_b = ms_b / max(nb, 1)
    achieved_tf = flops_launch / (avg_b * 1e-3) / 1e12
    nc, ms_c = prof["contract"]
    avg_c = ms_c / max(nc, 1)
    esz = 16 if dts == "c128" else 8
    bytes_in = 2 * 144 * esz * V * T * len(items)

    # HBM bytes per launch from rocprofv3 counters (profiles/traffic.json), valid
    # only while the kernel sources are the ones the counters were taken on
    traffic = {"blocks": None, "contract": None}
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tfile):
        ent = json.load(open(tfile)).get(args.workload, {})
        if ent.get("source_hash") == kernel_source_hash() and ent.get("precision") == prec:
            for k in traffic:
                traffic[k] = ent.get(k, {}).get("bytes_per_launch")
    # term sum: 6A + 2 FP64 flops per term and time slice, FP64 vector ALU peak
    # (256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz = 78.6 TFLOP/s)
    sum_flops = sum(plans[n].n_terms * T * (6 * plans[n].A + 2) for n, _ in items)
    sum_tf = sum_flops / (avg_c * 1e-3) / 1e12 if nc else 0.0
    roof_blocks = {"bound": "mfma", "kernel": "blocks_nucleon_kernel", "achieved": achieved_tf,
                   "peak": PEAK_TFLOPS[prec], "peak_name": PEAK_NAME[prec], "unit": "TFLOP/s",
                   "frac": achieved_tf / PEAK_TFLOPS[prec], "traffic": traffic["blocks"],
                   "flops_per_launch": flops_launch, "avg_launch_ms": avg_b}
    roof_sum = {"bound": "alu", "kernel": "contract_tg_kernel" if single else "contract_batch_kernel",
                "achieved": sum_tf, "peak": 78.6, "peak_name": "FP64 vector ALU", "unit": "TFLOP/s",
                "frac": sum_tf / 78.6, "traffic": traffic["contract"], "flops_per_launch": sum_flops,
                "avg_launch_ms": avg_c}
    dominant = roof_blocks if avg_b >= avg_c else roof_sum

    desc = ", ".join(f"{sum(1 for m, _ in items if m == n)}x {n}" for n in nuclei)
    out = {
        "metric": METRIC,
        "value": n_term_evals / step_s,
        "unit": "Wick terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * step_s,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "p64" else {"p32": "f32", "pb3": "bf16x3", "pb6": "bf16x6"}[prec],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc} on {X}x{Y}x{Z}x{T}, {dts} propagators, {prec} blocks "
                               f"+ FP64 term sum, all {T} time slices, {n_cfg} configuration(s)"
                               + ("" if single else ", one graph-captured batch"),
                   "lattice": [X, Y, Z, T], "n_cfg": n_cfg, "storage": dts, "precision": prec,
                   "correlators": len(items), "nuclei": {n: {"A": plans[n].A, "kinds": plans[n].n_kinds,
                                                             "terms": plans[n].n_terms} for n in nuclei}},
        "roofline": dominant,
        "rooflines": {"blocks": roof_blocks, "term_sum": roof_sum},
        "blocks_per_s": sum(plans[n].n_kinds * T for n, _ in items) / step_s,
        "block_tflops_gemm_equivalent": gemm_equiv / (avg_b * 1e-3) / 1e12,
        "terms_per_s_contract_kernel": n_term_evals / (avg_c * 1e-3) if nc else None,
        "kernel_ms": {k: (v[1] / v[0] if v[0] else None) for k, v in prof.items()},
        "propagator_GBs_blocks_kernel": bytes_in / (avg_b * 1e-3) / 1e9,
        "batch_timing": graph_ms,
        "plan_s": t_plan,
        "autotune_s": t_tune if not args.no_autotune else None,
        "input_gen_s": t_gen,
    }
    if single and prec == "p64" and not args.no_split:
        out["split_precision"] = split_precision(W, pl, step, B, C, args.steps, flops_launch)
    if single and not args.no_truncation:
        note("important-term truncation")
        out["important_terms"] = important_terms(W, pl, B, C, args.steps, wid, dims, dts, prec,
                                                 not args.no_autotune)
    if not args.no_cpu_baseline:
        note("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(items, nuclei, hu, hd, plans, C.cpu().numpy())
    print(json.dumps(out))


def gevp_bench(args):
    """Correlation matrix of three deuteron operators (Eqs. E1-E3): blocks of the
    matrix's kinds and the union term sum per step; beside it, the nine elements
    as nine separate correlators (one batched call)."""
    import torch
    import paper_2411_08962_amd as W
    desc, dims, wid = GEVP_WORKLOADS[args.workload]
    X, Y, Z, T = dims
    V = X * Y * Z
    names = ["2H", "2H-", "2H0"]
    n = len(names)
    hu, hd = gen_inputs(wid, 1, dims, np.complex128)
    du, dd = torch.from_numpy(hu).cuda(), torch.from_numpy(hd).cuda()
    t0 = time.time()
    g = W.gevp_plan_std(names)
    t_plan = time.time() - t0
    info = g.info()
    bp = g.blocks_plan()
    B = torch.empty((1, T, info["n_kinds"], W.BLOCK_LEN, 2), dtype=torch.float64, device="cuda")
    C = torch.empty((1, T, n, n, 2), dtype=torch.float64, device="cuda")

    def step():
        W.blocks(bp, du, dd, out=B)
        W.gevp_contract(g, B, out=C)

    elems = [W.plan_std_pair(names[i], names[j]) for i in range(n) for j in range(n)]
    Ce = torch.empty((n * n, T, 2), dtype=torch.float64, device="cuda")

    def step_elements():
        W.correlator(elems, [(e, 0) for e in range(n * n)], du, dd, use_graph=True, out=Ce)

    def timed(f):
        for _ in range(args.warmup):
            f()
        torch.cuda.synchronize()
        W.profile(True)
        t = time.perf_counter()
        for _ in range(args.steps):
            f()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / args.steps
        W.profile(False)
        return dt

    dt = timed(step)
    prof = {k: W.profile_read(k) for k in ("blocks", "blocks_reduce", "gevp_contract")}
    dt_e = timed(step_elements)
    Cm = C.cpu().numpy()[0]
    Cs = Ce.cpu().numpy()
    dev = max(abs(complex(*Cm[t, i, j]) - complex(*Cs[i * n + j, t])) / max(abs(complex(*Cs[i * n + j, t])), 1e-300)
              for i in range(n) for j in range(n) for t in range(T))
    nb, msb = prof["blocks"]
    nc, msc = prof["gevp_contract"]
    avg_b, avg_c = msb / max(nb, 1), msc / max(nc, 1)
    flops_b = block_flops_per_site("2H") * info["n_kinds"] / KINDS["2H"] * V * T
    tf_b = flops_b / (avg_b * 1e-3) / 1e12
    E = n * n
    sum_flops = info["n_terms"] * T * (6 * (info["A"] - 1) + 4 * E)
    tf_c = sum_flops / (avg_c * 1e-3) / 1e12
    roof_b = {"bound": "mfma", "kernel": "blocks_nucleon_kernel", "achieved": tf_b, "peak": 78.6,
              "peak_name": "FP64 MFMA", "unit": "TFLOP/s", "frac": tf_b / 78.6, "traffic": None,
              "flops_per_launch": flops_b, "avg_launch_ms": avg_b}
    roof_c = {"bound": "alu", "kernel": "gevp_contract_kernel", "achieved": tf_c, "peak": 78.6,
              "peak_name": "FP64 vector ALU", "unit": "TFLOP/s", "frac": tf_c / 78.6, "traffic": None,
              "flops_per_launch": sum_flops, "avg_launch_ms": avg_c}
    out = {
        "metric": METRIC,
        "value": info["n_element_terms"] * T / dt,
        "unit": "Wick terms/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {n}x{n} correlation matrix of {desc} on {X}x{Y}x{Z}x{T}, c128, "
                               f"FP64, all {T} time slices; value = element-table terms covered per second",
                   "lattice": [X, Y, Z, T], "plan": info, "plan_s": t_plan},
        "roofline": roof_b if avg_b >= avg_c else roof_c,
        "rooflines": {"blocks": roof_b, "union_term_sum": roof_c},
        "elementwise": {"ms_per_step": 1e3 * dt_e, "how": f"{n * n} element plans as one batched correlator call "
                                                          f"(graph), each element with its own blocks",
                        "speedup_of_union": dt_e / dt, "max_rel_diff_vs_union": float(dev)},
        "kernel_ms": {"blocks": avg_b, "gevp_contract": avg_c},
    }
    if not args.no_cpu_baseline:
        note("cpu baseline (oracle, element by element)")
        import oracle
        from oracle import operators as ops
        sys.path.insert(0, ROOT)
        from tests.helpers import gevp_element
        op_list = [ops.deuteron(+1), ops.deuteron(-1), ops.deuteron(0)]
        t0 = time.perf_counter()
        done = 0
        for t in range(T):
            for i in range(n):
                for j in range(n):
                    el = gevp_element(op_list, i, j)
                    oracle.sum_dp(el, oracle.blocks_raw(el, hu[0, t], hd[0, t]))
            done += 1
            if time.perf_counter() - t0 > 10.0:
                break
        dsec = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": info["n_element_terms"] * done / dsec, "unit": "Wick terms/s",
                               "cores": oracle.threads(), "kind": "oracle",
                               "sample": f"{done} time slices x {n * n} elements: oracle blocks + subset-DP term sum",
                               "seconds": dsec}
    print(json.dumps(out))


def point_bench(args):
    """Point-sink correlator by determinants (Eq. 2.9, App. A): all time slices
    of one configuration per step, FP64."""
    import torch
    import paper_2411_08962_amd as W
    nucleus, dims, wid = POINT_WORKLOADS[args.workload]
    X, Y, Z, T = dims
    V = X * Y * Z
    t0 = time.time()
    hu, hd = gen_inputs(wid, 1, dims, np.complex128)
    du, dd = torch.from_numpy(hu).cuda(), torch.from_numpy(hd).cuda()
    pp = W.point_plan_std(nucleus)
    info = pp.info()
    note(f"inputs and plan {time.time() - t0:.1f} s")
    C = torch.empty((1, T, 2), dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        W.point_correlator(pp, du, dd, out=C)
    torch.cuda.synchronize()
    W.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        W.point_correlator(pp, du, dd, out=C)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    W.profile(False)
    prof = {k: W.profile_read(k) for k in ("point_minors", "point_pairs", "point_reduce")}
    step_s = dt / args.steps
    pairs = info["n_sink_groups"] * info["n_src_groups"]
    slots = V * T
    # algorithmic flops per site-slice: minors by Laplace expansion (8 per complex
    # multiply-add), and 14 per determinant pair (two complex products and an add)
    f_u = info["n_rows_u"] * laplace_cmacs(info["n_u"]) * 8
    f_d = info["n_rows_d"] * laplace_cmacs(info["n_d"]) * 8
    f_p = pairs * 14
    ms = {k: (v[1] / v[0] if v[0] else None) for k, v in prof.items()}
    # per step the pairs kernel runs once per chunk: its total time per step
    t_pairs = prof["point_pairs"][1] / args.steps * 1e-3
    t_minors = prof["point_minors"][1] / args.steps * 1e-3
    tf_pairs = (f_u + f_p) * slots / t_pairs / 1e12
    tf_minors = f_d * slots / t_minors / 1e12
    roof_pairs = {"bound": "alu", "kernel": "pt_pairs_kernel", "achieved": tf_pairs, "peak": 78.6,
                  "peak_name": "FP64 vector ALU", "unit": "TFLOP/s", "frac": tf_pairs / 78.6, "traffic": None,
                  "flops_per_step": (f_u + f_p) * slots, "ms_per_step": t_pairs * 1e3,
                  "avg_launch_ms": ms["point_pairs"], "launches_per_step": prof["point_pairs"][0] / args.steps}
    roof_minors = {"bound": "alu", "kernel": "pt_minors_kernel", "achieved": tf_minors, "peak": 78.6,
                   "peak_name": "FP64 vector ALU", "unit": "TFLOP/s", "frac": tf_minors / 78.6, "traffic": None,
                   "flops_per_step": f_d * slots, "ms_per_step": t_minors * 1e3, "avg_launch_ms": ms["point_minors"]}
    out = {
        "metric": METRIC,
        "value": pairs * slots / step_s,
        "unit": "Wick terms/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * step_s,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: point-sink {nucleus} (all quarks of the sink at one site, summed "
                               f"over sites) by determinants on {X}x{Y}x{Z}x{T}, c128 propagators, FP64, all {T} "
                               f"time slices; a term is one (sink group, source group) pair of the weighted "
                               f"double sum at one site",
                   "lattice": [X, Y, Z, T], "nucleus": nucleus, "plan": info,
                   "dets_per_site": {"u": info["n_rows_u"] * info["n_cols_u"], "d": info["n_rows_d"] * info["n_cols_d"]}},
        "roofline": roof_pairs if t_pairs >= t_minors else roof_minors,
        "rooflines": {"pairs": roof_pairs, "minors": roof_minors},
        "s_per_time_slice": step_s / T,
        "paper_s_per_time_slice_24cubed": PAPER_POINT_24.get(nucleus),
        "kernel_ms": ms,
    }
    if nucleus in ("2H", "3He"):
        # the same correlator in the block form (per-site blocks and the plane-wave table)
        pl = W.plan_std(nucleus)
        Cb = torch.empty_like(C)
        for _ in range(max(args.warmup, 1)):
            W.point_blocks_correlator(pl, du, dd, out=Cb)
        torch.cuda.synchronize()
        W.profile(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            W.point_blocks_correlator(pl, du, dd, out=Cb)
        torch.cuda.synchronize()
        dtb = (time.perf_counter() - t0) / args.steps
        W.profile(False)
        nb, msb = W.profile_read("point_site_blocks")
        nc, msc = W.profile_read("contract")
        A, K, N = pl.info()
        nw = sum(len(pl.kind(k)[1]) for k in range(K))
        # per site: 28 flops per (block entry, weight) of the block build, 6A + 2 per term
        tf_b = 792 * nw * 28 * slots / (msb / args.steps * 1e-3) / 1e12
        tf_c = N * (6 * A + 2) * slots / (msc / args.steps * 1e-3) / 1e12
        cb, cd = Cb.cpu().numpy()[0], C.cpu().numpy()[0]
        dev = np.max(np.abs((cb[:, 0] - cd[:, 0]) + 1j * (cb[:, 1] - cd[:, 1])) / np.abs(cd[:, 0] + 1j * cd[:, 1]))
        out["block_form"] = {"ms_per_step": 1e3 * dtb, "s_per_time_slice": dtb / T, "speedup_vs_determinants": step_s / dtb,
                             "table_terms": N, "terms_per_s": N * slots / dtb,
                             "site_blocks_kernel": {"ms_per_step": msb / args.steps, "TFLOPs": tf_b, "frac_fp64_alu": tf_b / 78.6},
                             "term_sum": {"kernel": "contract_tg_kernel", "ms_per_step": msc / args.steps, "TFLOPs": tf_c,
                                          "frac_fp64_alu": tf_c / 78.6},
                             "max_rel_diff_vs_determinants": float(dev)}
    if not args.no_cpu_baseline:
        note("cpu baseline (oracle point route)")
        import oracle
        from oracle import operators as ops
        op = ops.by_name(nucleus)
        su = hu[0].reshape(T, V, 12, 12)
        sd = hd[0].reshape(T, V, 12, 12)
        Cg = C.cpu().numpy()[0]
        t0 = time.perf_counter()
        n_done, diffs = 0, []
        # whole time slices while the budget lasts, else a prefix of sites of slice 0
        for x in range(V):
            Br = oracle.blocks_raw(op, su[0, x:x + 1], sd[0, x:x + 1])
            oracle.sum_dp(op, Br)
            n_done += 1
            if time.perf_counter() - t0 > 10.0:
                break
        dsec = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": pairs * n_done / dsec, "unit": "Wick terms/s", "cores": oracle.threads(),
                               "kind": "oracle",
                               "sample": f"{n_done} sites of time slice 0: one-site blocks + subset-DP term sum per "
                                         f"site (the oracle's point-sink route); value = determinant pairs covered "
                                         f"per second", "seconds": dsec}
        if n_done == V:
            ref = op.scale * sum(oracle.sum_dp(op, oracle.blocks_raw(op, su[0, x:x + 1], sd[0, x:x + 1]))
                                 for x in range(V))
            out["cpu_baseline"]["gpu_vs_oracle_rel_diff_t0"] = float(abs(Cg[0, 0] + 1j * Cg[0, 1] - ref) / abs(ref))
    print(json.dumps(out))


def important_terms(W, pl, B, C, steps, wid, dims, dts, prec, tune):
    """Important-term truncation (Sec. 5, App. D): terms chosen once on blocks of
    a 2^3 calibration lattice (separate seed, up to 8 time slices), then the
    truncated table's term sum timed on the workload's blocks and its C(t)
    compared with the full table's."""
    import torch
    import wick_inputs as wi
    T = dims[3]
    ts = list(range(0, T, max(1, T // 8)))[:8]
    cu = torch.from_numpy(np.stack([wi.propagator(wid + 500, 0, 0, (2, 2, 2, T), t_slices=ts)])).cuda()
    cd = torch.from_numpy(np.stack([wi.propagator(wid + 500, 0, 1, (2, 2, 2, T), t_slices=ts)])).cuda()
    Bcal = W.blocks(pl, cu, cd).cpu()
    Cf = C.cpu().numpy()
    Cf = Cf[..., 0] + 1j * Cf[..., 1]
    res = []
    for keep in (0.1, 0.01):
        t0 = time.time()
        tp, dropped = pl.truncate(Bcal, keep)
        t_sel = time.time() - t0
        if tune:
            W.autotune(tp, dims, dts, prec)
        Ct = torch.empty_like(C)
        W.contract(tp, B, out=Ct)
        torch.cuda.synchronize()
        W.profile(True)
        for _ in range(steps):
            W.contract(tp, B, out=Ct)
        torch.cuda.synchronize()
        W.profile(False)
        n, ms = W.profile_read("contract")
        avg = ms / max(n, 1)
        ct = Ct.cpu().numpy()
        ct = ct[..., 0] + 1j * ct[..., 1]
        dev = np.abs(ct - Cf) / np.maximum(np.abs(Cf), 1e-300)
        res.append({"keep_fraction": keep, "n_terms": tp.n_terms, "select_s": t_sel,
                    "contract_ms": avg, "terms_per_s_contract_kernel": tp.n_terms * B.shape[0] * T / (avg * 1e-3),
                    "max_rel_dev_vs_full": float(dev.max()), "median_rel_dev_vs_full": float(np.median(dev)),
                    "calibration_dropped_weight_max": float(dropped.max())})
    return {"calibration": f"2x2x2 lattice, time slices {ts}, seed of workload {wid + 500}, p64 blocks",
            "note": "synthetic propagators have no gauge structure, so the term values are not heavy-tailed "
                    "as in the paper's ensembles; the deviation shows the mechanics, not the physics",
            "fractions": res}


def table_magnitude(pl, Bc):
    """sum_n |coef_n prod_a B[kidx_{a,n}]| for blocks Bc [K, 792] (host, numpy)."""
    kidx, coef = pl.table()
    flat = Bc.reshape(-1)
    prod = np.abs(coef)
    for a in range(kidx.shape[0]):
        prod = prod * np.abs(flat[kidx[a].astype(np.int64)])
    return prod.sum()


def split_precision(W, pl, step, B64, C64, steps, flops_launch):
    """Each split mode timed like the FP64 step; its C(t) compared with the FP64
    GPU result, relative to sum_n |term_n| (the table with the FP64 blocks)."""
    import torch
    step("p64")
    torch.cuda.synchronize()
    Bh = B64.cpu().numpy()
    Bc = Bh[..., 0] + 1j * Bh[..., 1]
    mag = np.array([[table_magnitude(pl, Bc[c, t]) for t in range(Bc.shape[1])] for c in range(Bc.shape[0])])
    c64 = C64.cpu().numpy().copy()
    res = {}
    for prec in ("p32", "pb3", "pb6"):
        step(prec)
        torch.cuda.synchronize()
        note(f"split precision {prec}")
        W.profile(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            step(prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        W.profile(False)
        nb, msb = W.profile_read("blocks")
        cs = C64.cpu().numpy()
        err = np.abs((cs[..., 0] - c64[..., 0]) + 1j * (cs[..., 1] - c64[..., 1])) / mag
        avg = msb / max(nb, 1)
        res[prec] = {"ms_per_step": 1e3 * dt / steps, "blocks_kernel_ms": avg,
                     "block_tflops": flops_launch / (avg * 1e-3) / 1e12,
                     "mfma_peak_frac": flops_launch / (avg * 1e-3) / 1e12 / PEAK_TFLOPS[prec],
                     "wick_terms_per_s": pl.n_terms * Bc.shape[0] * Bc.shape[1] / (dt / steps),
                     "max_rel_err_vs_fp64": float(err.max()), "median_rel_err_vs_fp64": float(np.median(err)),
                     "meets_1e-8": bool(err.max() <= 1e-8)}
    step("p64")
    torch.cuda.synchronize()
    return res


def cpu_baseline(items, nuclei, hu, hd, plans, C_gpu):
    """The oracle (blocks + subset-DP term sum) on sampled (item, time slice) pairs."""
    import oracle
    from oracle import operators as ops
    T = hu.shape[1]
    done, diffs, evals = [], [], 0
    t0 = time.perf_counter()
    # (item, t) pairs in a fixed order until about 10 s of CPU work (or all of them)
    order = [(i, (5 + 7 * k) % T) for k in range(T) for i in range(len(items))]
    for i, t in order:
        n, cfg = items[i]
        op = ops.by_name(n)
        Braw = oracle.blocks_raw(op, hu[cfg, t].astype(np.complex128), hd[cfg, t].astype(np.complex128))
        c = op.scale * oracle.sum_dp(op, Braw)
        got = C_gpu[i if len(items) > 1 else cfg, t, 0] + 1j * C_gpu[i if len(items) > 1 else cfg, t, 1]
        diffs.append(abs(got - c) / max(abs(c), 1e-300))
        done.append((n, cfg, t))
        evals += plans[n].n_terms
        if time.perf_counter() - t0 > 10.0:
            break
    dt = time.perf_counter() - t0
    return {"value": evals / dt, "unit": "Wick terms/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{len(done)} (nucleus, configuration, time slice) triples of the same workload, first "
                      f"{done[:4]}: oracle blocks (direct sums) + subset-DP term sum; value = table terms "
                      f"covered per second",
            "seconds": dt, "gpu_vs_oracle_max_rel_diff_of_C": float(max(diffs)),
            "same_table_numpy": same_table_cpu(plans[items[0][0]])}


def same_table_cpu(pl):
    """The deduplicated table itself evaluated on the host, on random blocks of
    the plan's shape: with numpy on one thread, and with the oracle's C loop on
    all threads (the method on the CPU, beside the oracle's own route)."""
    import oracle
    kidx, coef = pl.table()
    if kidx.shape[1] == 0:
        return None
    rng = np.random.default_rng(0)
    flat = (rng.standard_normal(pl.n_kinds * 792) + 1j * rng.standard_normal(pl.n_kinds * 792))
    idx = [k.astype(np.int64) for k in kidx]
    reps, t0 = 0, time.perf_counter()
    while True:
        prod = coef * flat[idx[0]]
        for a in range(1, len(idx)):
            prod *= flat[idx[a]]
        prod.sum()
        reps += 1
        if time.perf_counter() - t0 > 3.0:
            break
    dt = time.perf_counter() - t0
    sets = np.stack([flat] * 8)
    reps_c, t0 = 0, time.perf_counter()
    while True:
        oracle.table_sum(kidx, coef, sets)
        reps_c += 8
        if time.perf_counter() - t0 > 3.0:
            break
    dtc = time.perf_counter() - t0
    return {"value": reps * kidx.shape[1] / dt, "unit": "Wick terms/s", "threads": 1,
            "sample": f"{reps} evaluation(s) of the {kidx.shape[1]}-term table with numpy",
            "all_threads": {"value": reps_c * kidx.shape[1] / dtc, "threads": oracle.threads(),
                            "sample": f"{reps_c} evaluation(s) of the table by a C loop (OpenMP)"}}


if __name__ == "__main__":
    main()
