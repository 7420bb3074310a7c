"""Benchmark: NESA matrix-vector product throughput on one MI355X.

Workload: PEC sphere of radius 4 wavelengths, geodesic icosphere of frequency
82 (134,480 triangles, 201,720 RWG unknowns), leaf boxes of 0.25 wavelength
(levels 2..5), equivalent sources per box from the excess-bandwidth rule
(d0 = 3: Q = 441, 196, 81, 49), complex64 arithmetic, one right-hand side.
A step is one NESA product y = Z_NESA x (near field, radiation, source
transfer, translation, potential transfer, reception) with x and y resident
in HBM, in the canonical RWG order.

Prints one JSON line: the throughput, the roofline of the dominant stage, the
per-stage durations, a plain GMRES run on the same operator and the timed
CPU oracle on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12          # B/s
PEAK_FP32 = 157.3e12       # FLOP/s, dense FP32 matrix cores (and packed FP32 vector)
PEAK_BF16 = 2.5e15


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--nu", type=int, default=82, help="icosphere frequency (82: 201,720 unknowns)")
    p.add_argument("--radius", type=float, default=4.0)
    p.add_argument("--precision", default="c64", choices=["c64", "c128", "split"])
    p.add_argument("--nrhs", type=int, default=1)
    p.add_argument("--gmres-iters", type=int, default=300)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample-leaves", type=int, default=24)
    return p.parse_args()


def algorithmic(info, Q, esize):
    """Algorithmic bytes / flops of each phase of one product (nrhs = 1)."""
    n = info["n_rwg"]
    nl = info["L"] - info["l0"] + 1
    QL = Q[-1]
    nleaf = info["n_box"][-1]
    ph = {}
    # near field + reception (fused kernel): near blocks, V read once, x read, y written, o read
    ph["near_recv"] = {"bytes": info["near_entries"] * esize + n * 4 * QL * esize + 2 * n * esize
                       + nleaf * 4 * QL * esize,
                       "flops": 8 * info["near_entries"] + 8 * 4 * QL * n}
    ph["radiate"] = {"bytes": n * 4 * QL * esize + n * esize + nleaf * 4 * QL * esize,
                     "flops": 8 * 4 * QL * n}
    up = 0
    for i in range(1, nl):
        up += info["n_box"][i] * 8 * 4 * Q[i - 1] * Q[i]
    ph["upward"] = {"flops": up, "bytes": sum(info["n_box"][i] * 4 * Q[i] * esize for i in range(nl))}
    ph["downward"] = dict(ph["upward"])
    tflops = sum(8 * 4 * info["n_pairs"][i] * Q[i] * Q[i] for i in range(nl))
    tbytes = sum(min(info["n_pairs"][i], 316) * Q[i] * Q[i] * esize for i in range(nl))
    ph["translate"] = {"flops": tflops, "bytes": tbytes}
    return ph


def cpu_baseline(v, t, sample_leaves, seed=0):
    """Time the FP64 oracle's stages on a bounded sample of the same workload and
    extrapolate to one full product.  Sample: `sample_leaves` random leaves for the
    near field, radiation and reception; 32 random boxes per level for the
    translations and the transfers (operators built untimed)."""
    from threadpoolctl import threadpool_limits
    from oracle import nesa as onesa

    with threadpool_limits(limits=1):
        t_setup = time.perf_counter()
        ref = onesa.NesaOracle(v, t, leaf=0.25, d0=3, tau=1e-8)
        tr = ref.t
        rng = np.random.default_rng(seed)
        L, l0 = tr.L, tr.l0
        nleaf = len(tr.boxes[L])
        leaves = rng.choice(nleaf, size=min(sample_leaves, nleaf), replace=False)
        x = np.asarray(rng.standard_normal(ref.m.n) + 1j * rng.standard_normal(ref.m.n))
        for a in leaves:
            ref.near_block(a)
            ref.V(a)
        s = {l: [rng.standard_normal((4, ref.Q[l])) + 0j for _ in tr.boxes[l]] for l in ref.levels}
        for l in ref.levels:
            for off in {(tuple(np.subtract(tr.boxes[l][a], tr.boxes[l][b]))) for a in range(len(tr.boxes[l]))
                        for b in tr.il[l][a]}:
                ref.D(l, off)
        for l in range(l0 + 1, L + 1):
            for o in range(8):
                ref.C(l, o)
        t_setup = time.perf_counter() - t_setup
        est = {}
        # near field (Eq. 9) and radiation / reception (Eq. 10, 14) per leaf
        t0 = time.perf_counter()
        for a in leaves:
            rows, cols, Z = ref.near_block(a)
            _ = Z @ x[cols]
        est["near"] = (time.perf_counter() - t0) / len(leaves) * nleaf
        t0 = time.perf_counter()
        for a in leaves:
            _ = ref.V(a) @ x[tr.leaf_rwgs[a]]
            _ = np.einsum("c,cqn,cq->n", ref.w, ref.V(a), s[L][0])
        est["radiate_receive"] = (time.perf_counter() - t0) / len(leaves) * nleaf
        # translations (Eq. 12) per level
        tt = 0.0
        for l in ref.levels:
            nb = len(tr.boxes[l])
            boxes = rng.choice(nb, size=min(32, nb), replace=False)
            t0 = time.perf_counter()
            for a in boxes:
                ref.translate(s, l, a)
            tt += (time.perf_counter() - t0) / len(boxes) * nb
        est["translate"] = tt
        # transfers (Eq. 11, 13)
        tt = 0.0
        for l in range(l0 + 1, L + 1):
            nb = len(tr.boxes[l])
            boxes = rng.choice(nb, size=min(32, nb), replace=False)
            t0 = time.perf_counter()
            for b in boxes:
                C = ref.C(l, ref.octant(l, b))
                _ = (C @ s[l][b].T).T
                _ = (C.T @ s[l - 1][tr.parent[l][b]].T).T
            tt += (time.perf_counter() - t0) / len(boxes) * nb
        est["transfer"] = tt
    total = sum(est.values())
    return {"value": ref.m.n / total / 1e6, "unit": "Munknowns*matvec/s", "cores": 1, "kind": "oracle",
            "sample": ("FP64 NumPy oracle, one thread: near field and radiation/reception timed on %d random "
                       "leaves of %d, translations and transfers on 32 random boxes per level; per-stage "
                       "means scaled to the full tree (extrapolated %.2f s per product; operators built "
                       "untimed in %.1f s)" % (len(leaves), nleaf, total, t_setup)),
            "stage_seconds": {k: round(v_, 3) for k, v_ in est.items()}}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: there is no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    from paper_1801_03589_amd import nesa

    prec = {"c64": nesa.C64, "c128": nesa.C128, "split": nesa.C64_SPLIT}[args.precision]
    esize = 16 if prec == nesa.C128 else 8
    dt = torch.complex128 if prec == nesa.C128 else torch.complex64
    setup = {}
    t0 = time.perf_counter()
    v, t = synth.icosphere(args.nu, args.radius)
    tree = nesa.build_tree(v, t, 0.25)
    info = tree.info()
    setup["tree_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    near = nesa.assemble_near(tree)
    setup["near_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    far = nesa.assemble_translations(tree, d0=3, tau=1e-8)
    setup["far_s"] = time.perf_counter() - t0
    nl = info["L"] - info["l0"] + 1
    Q = [int(q) for q in far.q(nl)]
    t0 = time.perf_counter()
    op = nesa.op_create(tree, near, far, prec)
    setup["upload_s"] = time.perf_counter() - t0
    n = info["n_rwg"]
    x = torch.from_numpy(synth.complex_normal(n, 0)).to(dt).cuda()
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        nesa.matvec(op, x, y, stream=stream)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        nesa.matvec(op, x, y, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / args.steps
    value = n / (ms * 1e-3) / 1e6
    # per-stage and per-launch durations (hipEvents on the launch stream), averaged
    xl = torch.empty_like(x)
    yl = torch.empty_like(x)
    reps = 5
    pm = np.zeros(5)
    launches = None
    for _ in range(reps):
        pm += nesa.matvec_phase_times(op, xl.copy_(x), yl, stream=stream)
        lt = nesa.matvec_launch_times(op, xl, yl, stream=stream)
        if launches is None:
            launches = [[k, l, 0.0] for k, l, _ in lt]
        for i, (_, _, m) in enumerate(lt):
            launches[i][2] += m / reps
    pm /= reps
    names = ["radiate", "upward", "translate", "downward", "near_recv"]
    phase_ms = {k: round(float(pm[i]), 4) for i, k in enumerate(names)}
    alg = algorithmic(info, Q, esize)
    l0 = info["l0"]
    kern = {}
    for kind, lev, m in launches:
        e = kern.setdefault(kind, {"ms": 0.0, "launches": 0, "flops": 0.0, "bytes": 0.0})
        e["ms"] += m
        e["launches"] += 1
        i = lev - l0
        if kind in ("translate_gemm", "translate_fp64"):
            e["flops"] += 8 * 4 * info["n_pairs"][i] * Q[i] * Q[i]
        elif kind in ("upward_gemm", "downward_gemm", "upward_fp64", "downward_fp64"):
            e["flops"] += info["n_box"][i] * 8 * 4 * Q[i - 1] * Q[i]
        elif kind == "near_recv":
            e["bytes"] += alg["near_recv"]["bytes"]
            e["flops"] += alg["near_recv"]["flops"]
        elif kind == "radiate":
            e["bytes"] += alg["radiate"]["bytes"]
            e["flops"] += alg["radiate"]["flops"]
        elif kind in ("translate_sum",):
            e["bytes"] += 2 * info["n_pairs"][i] * 4 * Q[i] * esize
        elif kind in ("upward_sum",):
            e["bytes"] += 2 * info["n_box"][i] * 4 * Q[i - 1] * esize
    dom = max(kern, key=lambda k: kern[k]["ms"])
    kd = kern[dom]
    sec = kd["ms"] * 1e-3
    if kd["bytes"] == 0 or dom.endswith("gemm") or dom.endswith("fp64"):
        peak = PEAK_FP32 if prec != nesa.C128 else 78.6e12
        roof = {"bound": "mfma", "achieved": kd["flops"] / sec / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": kd["bytes"] / sec / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["kernel"] = {"translate_gemm": "k_translate_gemm", "near_recv": "k_near_recv",
                      "upward_gemm": "k_transfer_gemm", "downward_gemm": "k_transfer_gemm"}.get(dom, dom)
    roof["launches_per_product"] = kd["launches"]
    roof["avg_launch_ms"] = kd["ms"] / kd["launches"]
    kernels = {k: {"ms_per_product": round(v_["ms"], 4), "launches": v_["launches"],
                   "TFLOP/s": round(v_["flops"] / (v_["ms"] * 1e-3) / 1e12, 2) if v_["flops"] else None,
                   "GB/s": round(v_["bytes"] / (v_["ms"] * 1e-3) / 1e9, 1) if v_["bytes"] else None}
               for k, v_ in kern.items()}
    phases = {}
    for k in names:
        s_ = phase_ms[k] * 1e-3
        phases[k] = {"ms": phase_ms[k], "GB/s": round(alg[k]["bytes"] / s_ / 1e9, 1),
                     "TFLOP/s": round(alg[k]["flops"] / s_ / 1e12, 2)}
    # GMRES on the same operator (plain, restart 50, tolerance 1e-4)
    b = torch.empty_like(x)
    nesa.rhs_plane_wave(op, [0, 0, 1], [1, 0, 0], b, stream=stream)
    xs = torch.zeros_like(b)
    rc, rep, _ = nesa.gmres_solve(op, b, xs, restart=50, max_iters=args.gmres_iters, tol=1e-4,
                                  stream=stream)
    gm = {"plain_fp32": {"iters": rep[0]["iters"], "true_rel_residual": rep[0]["true_rel_residual"],
                         "seconds": round(rep[0]["seconds"], 3), "converged": rc == 0,
                         "max_iters": args.gmres_iters}}
    out = {
        "metric": "NESA matvec Munknowns/s",
        "value": round(value, 3),
        "unit": "Munknowns*matvec/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"c64": "complex64", "c128": "complex128", "split": "complex64+bf16x3"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "pec_sphere_r%gl_icosphere%d_%drwg" % (args.radius, args.nu, n),
                   "n_unknowns": n, "nrhs": 1, "leaf_lambda": 0.25, "levels": [info["l0"], info["L"]],
                   "Q": Q, "boxes": info["n_box"], "pairs": info["n_pairs"],
                   "near_entries": info["near_entries"], "parallelism": "single_gpu"},
        "roofline": roof,
        "phases": phases,
        "kernels": kernels,
        "wall_s_timed": round(wall, 4),
        "setup_s": {k: round(v_, 2) for k, v_ in setup.items()},
        "gmres": gm,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(v, t, args.cpu_sample_leaves)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
