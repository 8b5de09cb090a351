"""Benchmark of the hot path: blocks + Wick-term sum for every time slice.

One step = the baryon blocks of every kind on every time slice of every
configuration (HIP, MFMA) followed by the FP64 sum over the deduplicated term
table for every (configuration, time slice), i.e. one full C(t) set. Inputs are
seeded synthetic propagators, already resident in HBM when the timed region
starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--precision p64]

Workloads: batch64-16^3x32 (default: 64 complex64 configurations, 8 2H,
24 3He and 32 4He correlators in one graph-captured batch), 2H-4^3x8 (small
case), 3He-16^3x32, 4He-24^3x48, 7Li-32^3x64 (the 4He and 3H cluster
correlators, batched). ``value`` is the FP64 path; the split-precision modes
are timed beside it on the same inputs, and every precision's C(t) is
compared with the oracle on sampled (correlator, time slice) pairs. Prints
one JSON line. Only the oracle legs (``cpu_baseline`` and the sampled
reference values) use the oracle.
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
DEFAULT = "batch64-16^3x32"

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


def sum_flops_per_slice(plan):
    """FP64 flops of the term-sum kernel per time slice, from the plan's table
    (wick_plan_sum_work): 6A + 2 per term for the per-term forms; for the word
    forms 14 per two-leaf word (q0 b0 + q1 b1 with real q: 6, the complex
    multiply-add by the node entry: 8) and 10 per one-leaf word, plus per
    segment the complex product by its prefix (6 per prefix entry) or, in the
    factored form, by unit * G (2), and the complex multiply-add into the sum
    (8). A complex palette coefficient adds 8 flops per gathered leaf."""
    w = plan.sum_work()
    A = plan.A
    if w["form"] in ("plain", "packed"):
        return plan.n_terms * (6 * A + 2)
    per_seg = 10 if w["form"] == "factored" else 6 * (A - 2) + 8
    per2, per1 = (14, 10) if w["form"] != "segmented-palette" else (30, 18)
    return per2 * w["words2"] + per1 * w["words1"] + per_seg * w["segments"]


def gemm_flops_per_site(nucleus, kinds=None):
    """The MFMA contraction: 12 rows (i1) per kind x 144 columns x 3 E rows x 8
    flops per complex multiply-add (counted as written, whatever the number of
    real MFMAs a precision spends on one complex product)."""
    return 12 * (KINDS[nucleus] if kinds is None else kinds) * 144 * 3 * 8


def erow_flops_per_site(nucleus):
    """The E rows on the vector ALU: per nonzero diquark entry 6 complex products
    and adds for the three colour cross products (8 flops each) per column."""
    return sum(144 * npair * 6 * 8 for npair in EROWS[nucleus])


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
    ap.add_argument("--split", default=None,
                    help="comma-separated split modes timed beside the main precision (default: p32,pb6 for "
                         "batches, p32,pb3,pb6 for single correlators; 'none' for none)")
    ap.add_argument("--samples", type=int, default=8, help="(correlator, time slice) pairs checked by the oracle")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip every oracle leg")
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
    single = len(items) == 1
    if args.no_split or args.split == "none":
        splits = []
    elif args.split:
        splits = [p for p in args.split.split(",") if p and p != prec]
    else:
        splits = [p for p in (("p32", "pb3", "pb6") if single else ("p32", "pb6")) if p != prec]
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
            for p in [prec] + splits:
                W.autotune(plans[n], dims, dts, p)
        t_tune = time.time() - t0
        note(f"autotune {t_tune:.1f} s")
    if single:
        pl = plans[nuclei[0]]
        A, K, N = pl.info()
        B = torch.empty((n_cfg, T, K, W.BLOCK_LEN, 2), dtype=torch.float64, device="cuda")
        C = torch.empty((n_cfg, T, 2), dtype=torch.float64, device="cuda")

        def step(p, graph=True):
            W.blocks(pl, du, dd, p, out=B)
            W.contract(pl, B, out=C)
    else:
        plist = [plans[n] for n in nuclei]
        bitems = [(nuclei.index(n), c) for n, c in items]
        C = torch.empty((len(items), T, 2), dtype=torch.float64, device="cuda")

        def step(p, graph=True):
            W.correlator(plist, bitems, du, dd, p, use_graph=graph, out=C)

        if not args.no_autotune:
            # the batched launch tuned as a whole on these inputs (outside the timed region)
            t0 = time.time()
            for p in [prec] + splits:
                W.autotune_batch(plist, bitems, du, dd, p)
            t_tune += time.time() - t0
            note(f"batch autotune done ({t_tune:.1f} s of tuning in total)")

    runs = {}
    for p in [prec] + splits:
        runs[p] = timed_steps(W, torch, step, p, single, C, args.steps, args.warmup)
        note(f"{p}: {runs[p]['ms_per_step']:.3f} ms/step")

    n_term_evals = sum(plans[n].n_terms * T for n, _ in items)
    slice_flops = {n: sum_flops_per_slice(plans[n]) for n in plans}
    traffic = load_traffic(args.workload)

    def rooflines(p, r):
        prof = r["prof"]
        nb, ms_b = prof["blocks"]
        nc, ms_c = prof["contract"]
        avg_b, avg_c = ms_b / max(nb, 1), ms_c / max(nc, 1)
        gemm = sum(gemm_flops_per_site(n) * V * T for n, _ in items)
        erow = sum(erow_flops_per_site(n) * V * T for n, _ in items)
        tf_b = gemm / (avg_b * 1e-3) / 1e12
        # term sum: the flops of the table's words per time slice (sum_flops_per_slice),
        # FP64 vector ALU peak (256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz = 78.6 TFLOP/s)
        sum_flops = sum(slice_flops[n] * T for n, _ in items)
        tf_c = sum_flops / (avg_c * 1e-3) / 1e12 if nc else 0.0
        tr = traffic.get(p, {})
        rb = {"bound": "mfma", "kernel": "blocks_nucleon_kernel", "achieved": tf_b, "peak": PEAK_TFLOPS[p],
              "peak_name": PEAK_NAME[p], "unit": "TFLOP/s", "frac": tf_b / PEAK_TFLOPS[p],
              "traffic": tr.get("blocks"), "flops_per_launch": gemm, "avg_launch_ms": avg_b,
              "erow_valu_flops_per_launch": erow, "erow_valu_tflops": erow / (avg_b * 1e-3) / 1e12}
        if p in SPLIT_PRODUCTS:
            # one BF16 MFMA pass per limb product: the mode's own effective peak
            rb["frac_of_effective_peak"] = tf_b / (PEAK_TFLOPS[p] / SPLIT_PRODUCTS[p])
        rc = {"bound": "alu", "kernel": "contract_tg_kernel" if single else "contract_batch_kernel",
              "achieved": tf_c, "peak": 78.6, "peak_name": "FP64 vector ALU", "unit": "TFLOP/s",
              "frac": tf_c / 78.6, "traffic": tr.get("contract"), "flops_per_launch": sum_flops,
              "avg_launch_ms": avg_c}
        # the flat count, 6A + 2 flops per deduplicated term and time slice: what a
        # per-term evaluation would execute; above the peak when the table's words
        # share sub-sums (the factored form), so a rate of the method, not of the ALU
        flat = sum(plans[n].n_terms * T * (6 * plans[n].A + 2) for n, _ in items)
        if nc:
            rc["flat_6A2_flops_per_launch"] = flat
            rc["flat_6A2_tflops"] = flat / (avg_c * 1e-3) / 1e12
            rc["flat_6A2_over_fp64_alu_peak"] = rc["flat_6A2_tflops"] / 78.6
        return rb, rc

    main_run = runs[prec]
    rb, rc = rooflines(prec, main_run)
    step_s = main_run["ms_per_step"] * 1e-3
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
        "dtype": DTYPE_NAME[prec],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc} on {X}x{Y}x{Z}x{T}, {dts} propagators, {prec} blocks "
                               f"+ FP64 term sum, all {T} time slices, {n_cfg} configuration(s)"
                               + ("" if single else ", one graph-captured batch"),
                   "lattice": [X, Y, Z, T], "n_cfg": n_cfg, "storage": dts, "precision": prec,
                   "correlators": len(items), "nuclei": {n: {"A": plans[n].A, "kinds": plans[n].n_kinds,
                                                             "terms": plans[n].n_terms} for n in nuclei}},
        "roofline": rb if rb["avg_launch_ms"] >= rc["avg_launch_ms"] else rc,
        "rooflines": {"blocks": rb, "term_sum": rc},
        "blocks_per_s": sum(plans[n].n_kinds * T for n, _ in items) / step_s,
        "block_tflops": rb["achieved"],
        "terms_per_s_contract_kernel": n_term_evals / (rc["avg_launch_ms"] * 1e-3) if rc["avg_launch_ms"] else None,
        "kernel_ms": main_run["kernel_ms"],
        "propagator_GBs_blocks_kernel": 2 * 144 * (16 if dts == "c128" else 8) * V * T * len(items)
                                        / (rb["avg_launch_ms"] * 1e-3) / 1e9,
        "batch_timing": main_run["graph"],
        "plan_s": t_plan,
        "autotune_s": t_tune if not args.no_autotune else None,
        "input_gen_s": t_gen,
    }
    split_out = {}
    for p in splits:
        r = runs[p]
        sb, sc = rooflines(p, r)
        split_out[p] = {"ms_per_step": r["ms_per_step"], "wick_terms_per_s": n_term_evals / (r["ms_per_step"] * 1e-3),
                        "speedup_vs_" + prec: main_run["ms_per_step"] / r["ms_per_step"],
                        "dtype": DTYPE_NAME[p], "kernel_ms": r["kernel_ms"], "batch_timing": r["graph"],
                        "rooflines": {"blocks": sb, "term_sum": sc},
                        "roofline": sb if sb["avg_launch_ms"] >= sc["avg_launch_ms"] else sc}
    if split_out:
        out["split_precision"] = split_out
    if not args.no_cpu_baseline:
        note("oracle: sampled reference values and the cpu baseline")
        samples = oracle_samples(items, plans, hu, hd, T, args.samples)
        errs = {p: errors_vs_oracle(samples, runs[p]["C"], items, single, TOL[p]) for p in runs}
        out["error_vs_oracle"] = {
            "what": "|dC| / sum_n |term_n| (sum over the deduplicated table with the oracle's blocks) and "
                    "|dC| / |C|, the oracle's C(t) from direct block sums and the subset-DP term sum",
            "samples": [{"item": s["item"], "nucleus": s["nucleus"], "cfg": s["cfg"], "t": s["t"]} for s in samples],
            **errs}
        out["cpu_baseline"] = cpu_baseline(samples, plans)
        if single and prec == "p64":
            out["cpu_baseline"]["same_table"] = same_table_cpu(plans[items[0][0]])
    if single and not args.no_truncation:
        note("important-term truncation")
        step(prec)
        torch.cuda.synchronize()
        out["important_terms"] = important_terms(W, pl, B, C, args.steps, wid, dims, dts, prec,
                                                 not args.no_autotune)
    print(json.dumps(out))


SPLIT_PRODUCTS = {"pb3": 3, "pb6": 6}
DTYPE_NAME = {"p64": "f64", "p32": "f32", "pb3": "bf16x3", "pb6": "bf16x6"}
# error bounds relative to sum_n |term_n|: FP64 blocks 1e-12, FP32 and three BF16
# limbs 1e-8 (the split bound); two BF16 limbs are measured against 1e-6
TOL = {"p64": 1e-12, "p32": 1e-8, "pb6": 1e-8, "pb3": 1e-6}
KERNELS = ("blocks", "blocks_reduce", "contract", "contract_finalize")


def timed_steps(W, torch, step, prec, single, C, steps, warmup):
    """Warm up, then time `steps` steps between device synchronisations; the
    per-kernel HIP-event durations come from the library's probes on the launch
    stream. A graph-captured batch cannot hold the probes' events, so its
    per-kernel durations come from the same batch launched eagerly afterwards."""
    for _ in range(warmup):
        step(prec)
    torch.cuda.synchronize()
    W.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step(prec)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    W.profile(False)
    Cg = C.cpu().numpy().copy()
    prof = {k: W.profile_read(k) for k in KERNELS}
    graph = None
    if not single:
        g = W.profile_read("correlator")
        step(prec, graph=False)
        torch.cuda.synchronize()
        W.profile(True)
        for _ in range(steps):
            step(prec, graph=False)
        torch.cuda.synchronize()
        W.profile(False)
        prof = {k: W.profile_read(k) for k in KERNELS}
        e = W.profile_read("correlator")
        graph = {"graph_launch_ms": g[1] / max(g[0], 1), "eager_batch_ms": e[1] / max(e[0], 1)}
    return {"ms_per_step": 1e3 * dt, "C": Cg, "prof": prof, "graph": graph,
            "kernel_ms": {k: (v[1] / v[0] if v[0] else None) for k, v in prof.items()}}


def load_traffic(workload):
    """HBM bytes per launch from rocprofv3 counters (profiles/traffic.json), per
    precision, valid only while the kernel sources hash to the recorded value."""
    out = {}
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(tfile):
        return out
    h = kernel_source_hash()
    for key, ent in json.load(open(tfile)).items():
        w, _, p = key.partition("|")
        if w == workload and ent.get("source_hash") == h:
            out[p] = {k: ent.get(k, {}).get("bytes_per_launch") for k in ("blocks", "contract")}
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def sample_pairs(items, T, n):
    """(item, t) pairs for the oracle: the nuclei in proportion to their share of
    the items, time slices spread over [0, T) and including the first and last."""
    by_nuc = {}
    for i, (nuc, _) in enumerate(items):
        by_nuc.setdefault(nuc, []).append(i)
    quota = {nuc: max(1, round(n * len(ix) / len(items))) for nuc, ix in by_nuc.items()}
    ts = [0, T - 1] + [(5 + 7 * k) % T for k in range(n)]
    out, k = [], 0
    for nuc, ix in by_nuc.items():
        for j in range(quota[nuc]):
            out.append((ix[j % len(ix)], ts[k % len(ts)]))
            k += 1
    return out


def compact_layout(B):
    """[..., 12, 12, 12] antisymmetric blocks -> [..., 792], entry pair(i1 < i3) * 12 + i2
    with pair(i1, i3) = i3 (i3 - 1) / 2 + i1 (the library's block layout)."""
    out = np.zeros(B.shape[:-3] + (792,), dtype=B.dtype)
    for i3 in range(12):
        for i1 in range(i3):
            out[..., (i3 * (i3 - 1) // 2 + i1) * 12:(i3 * (i3 - 1) // 2 + i1) * 12 + 12] = B[..., i1, :, i3]
    return out


def kind_order(op, pl):
    """For each kind of the plan, the oracle operator's kind with the same flavors and weights."""
    def canon(fl, w):
        return tuple(int(f) for f in fl), tuple(sorted((int(a), int(b), int(c), int(x), int(y)) for a, b, c, x, y in w))
    index = {}
    for i, k in enumerate(op.kinds):
        index.setdefault(canon(k.flavors, k.w), i)
    return [index[canon(*pl.kind(k))] for k in range(pl.n_kinds)]


def oracle_samples(items, plans, hu, hd, T, n):
    """The oracle's C(t) (direct block sums, subset-DP term sum; timed) and the
    error scale sum_n |term_n| (the plan's table with the oracle's blocks, Eq. 2.4
    form) on sampled (item, time slice) pairs."""
    import oracle
    from oracle import operators as ops
    tables = {}
    out = []
    for i, t in sample_pairs(items, T, n):
        nuc, cfg = items[i]
        op = ops.by_name(nuc)
        su, sd = hu[cfg, t].astype(np.complex128), hd[cfg, t].astype(np.complex128)
        t0 = time.perf_counter()
        ref = op.scale * oracle.sum_dp(op, oracle.blocks_raw(op, su, sd))
        dt = time.perf_counter() - t0
        pl = plans[nuc]
        if nuc not in tables:
            kidx, coef = pl.table()
            tables[nuc] = (kidx, np.abs(coef), kind_order(op, pl))
        kidx, acoef, order = tables[nuc]
        Bc = np.stack([compact_layout(oracle.block_eq24(op.kinds[k], su, sd)) for k in order])
        mag = float(oracle.table_sum(kidx, acoef, np.abs(Bc).reshape(1, -1))[0].real)
        out.append({"item": i, "nucleus": nuc, "cfg": cfg, "t": t, "C": ref, "mag": mag, "oracle_s": dt,
                    "n_terms": pl.n_terms})
    return out


def errors_vs_oracle(samples, C, items, single, tol):
    rel_terms, rel_c = [], []
    for s in samples:
        row = s["cfg"] if single else s["item"]
        got = C[row, s["t"], 0] + 1j * C[row, s["t"], 1]
        d = abs(got - s["C"])
        rel_terms.append(d / s["mag"])
        rel_c.append(d / max(abs(s["C"]), 1e-300))
    return {"max_dC_over_sum_terms": float(max(rel_terms)), "max_dC_over_C": float(max(rel_c)),
            "per_sample_dC_over_sum_terms": [float(v) for v in rel_terms],
            "per_sample_dC_over_C": [float(v) for v in rel_c],
            "bound": tol, "meets_bound": bool(max(rel_terms) <= tol)}


def cpu_baseline(samples, plans):
    """The oracle's own route (blocks by direct sums + subset-DP term sum) timed
    on the sampled (item, time slice) pairs; value = table terms covered per second."""
    import oracle
    dt = sum(s["oracle_s"] for s in samples)
    evals = sum(s["n_terms"] for s in samples)
    which = ", ".join("%s cfg %d t %d" % (s["nucleus"], s["cfg"], s["t"]) for s in samples)
    return {"value": evals / dt, "unit": "Wick terms/s", "cores": oracle.threads(), "cpu_model": cpu_model(),
            "kind": "oracle",
            "sample": f"{len(samples)} (nucleus, configuration, time slice) triples of the same workload "
                      f"({which}): oracle blocks "
                      f"(direct sums) + subset-DP term sum; value = deduplicated-table terms covered per second",
            "seconds": dt}


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
    flops_b = gemm_flops_per_site("2H", info["n_kinds"]) * V * T
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
        from oracle.operators import gevp_element
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
    if nucleus in ("2H", "3He", "4He"):
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
        # per site: 28 flops per (block entry, weight) of the block build; the term
        # sum's flops per slice from its table (sum_flops_per_slice)
        tf_b = 792 * nw * 28 * slots / (msb / args.steps * 1e-3) / 1e12
        tf_c = sum_flops_per_slice(pl) * slots / (msc / args.steps * 1e-3) / 1e12
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
