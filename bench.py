"""Benchmark: NESA matrix-vector product throughput on one MI355X.

Workload: PEC sphere of radius 4 wavelengths, geodesic icosphere of frequency
82 (134,480 triangles, 201,720 RWG unknowns), leaf boxes of 0.25 wavelength
(levels 2..5), equivalent sources per box from the excess-bandwidth rule
(d0 = 3: Q = 441, 196, 81, 49), complex64 arithmetic, one right-hand side.
A step is one NESA product y = Z_NESA x (near field, radiation, source
transfer, translation, potential transfer, reception) with x and y resident
in HBM, in the canonical RWG order.

Prints one JSON line: the throughput, the roofline of the dominant stage, the
per-stage durations, the time to a 1e-4 residual of GMRES(50) on the same
operator (plain, Schwarz-preconditioned and learned-preconditioned FGMRES),
the throughput of a batched product over several right-hand sides, and the
timed CPU oracle on a bounded sample.
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


def log(msg):
    """Progress on stderr (stdout carries the one JSON line)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--nu", type=int, default=82, help="icosphere frequency (82: 201,720 unknowns)")
    p.add_argument("--radius", type=float, default=4.0)
    p.add_argument("--precision", default="c64", choices=["c64", "c128", "split", "split_fp16"])
    p.add_argument("--nrhs", type=int, default=8, help="right-hand sides of the batched product line")
    p.add_argument("--gmres-iters", type=int, default=1500)
    p.add_argument("--only-product", action="store_true",
                   help="time the product only (no GMRES, batched or CPU lines): the profiled command")
    p.add_argument("--counters", action="store_true",
                   help="run 5 products and a 512 MiB device copy for hardware-counter passes, then exit")
    p.add_argument("--bodies", type=int, default=256,
                   help="uneven bodies in the batched-forest line (256: the full batch; 0: skip)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--only-model2d", action="store_true",
                   help="time only the 2D model problem (paper's own workload) and print its section")
    p.add_argument("--aircraft-nrhs", type=int, default=64,
                   help="incidences of the aircraft-like body's batched product (0: skip that line)")
    p.add_argument("--aircraft-fp32", action="store_true",
                   help="also time the aircraft's batched product with FP32 translations")
    p.add_argument("--only-aircraft", action="store_true", help="time only the aircraft-like body's line")
    p.add_argument("--only-learned-family", action="store_true",
                   help="run only the learned preconditioner on the aircraft family (held-out seed 999)")
    p.add_argument("--learned-bodies", type=int, default=8, help="training bodies of that line")
    p.add_argument("--only-schwarz", action="store_true",
                   help="time only the device setup of the Schwarz preconditioner on the bench sphere")
    return p.parse_args()


def algorithmic(info, Q, esize):
    """Algorithmic bytes / flops of each phase of one product (nrhs = 1)."""
    n = info["n_rwg"]
    nl = info["L"] - info["l0"] + 1
    QL = Q[-1]
    nleaf = info["n_box"][-1]
    ph = {}
    # near field (reciprocity half storage: blocks Z_ab with b >= a, read once;
    # the outputs Z_ab^T x_a written and read back) + reception: V read once,
    # x read, y written, o read; flops: one complex MAC per entry of the full
    # near field (each stored off-diagonal entry serves two)
    nt = info["near_transposed"]
    ph["near_recv"] = {"bytes": info["near_entries_half"] * esize + 2 * nt * esize + n * 4 * QL * esize
                       + 2 * n * esize + nleaf * 4 * QL * esize,
                       "flops": 8 * info["near_entries"] + 8 * 4 * QL * n}
    ph["radiate"] = {"bytes": n * 4 * QL * esize + n * esize + nleaf * 4 * QL * esize,
                     "flops": 8 * 4 * QL * n}
    # reception alone (the overlapped product adds it, with the transposed
    # near-field outputs, after the side-stream near field)
    ph["receive"] = {"bytes": n * 4 * QL * esize + 3 * n * esize + nleaf * 4 * QL * esize + nt * esize,
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(v, t, seed=0):
    """The FP64 oracle's whole product on the host: the NumPy oracle builds the
    tree, point sets and fitting operators; its C loop form (oracle/nesa_c.c,
    pinned against it) assembles the near blocks and radiation matrices
    (untimed) and runs the full product (near field and the five far-field
    stages), timed on every core this process may use and on one core.  The
    same 201,720-unknown operator (d0 = 3) as the GPU line."""
    from oracle import nesa as onesa
    from oracle import nesa_c

    t0 = time.perf_counter()
    ref = onesa.NesaOracle(v, t, leaf=0.25, d0=3, tau=1e-8)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    nesa_c.set_threads(cores)
    c = nesa_c.NesaC(ref)
    setup = time.perf_counter() - t0
    x = np.asarray(np.random.default_rng(seed).standard_normal(ref.m.n)
                   + 1j * np.random.default_rng(seed + 1).standard_normal(ref.m.n))
    times = {}
    for th in (cores, 1):
        nesa_c.set_threads(th)
        reps = 2 if th > 1 else 1
        best = None
        for _ in range(reps):
            t0 = time.perf_counter()
            c.matvec(x)
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        times[th] = best
        log("CPU oracle product on %d thread(s): %.2f s" % (th, best))
    n = ref.m.n
    return {"value": n / times[cores] / 1e6, "unit": "Munknowns*matvec/s", "cores": cores, "kind": "oracle",
            "sample": ("whole FP64 product (near field + five far-field stages) of the same 201,720-unknown "
                       "operator by the oracle's C loops with OpenMP, %d threads: %.2f s (best of 2); "
                       "operators assembled untimed in %.1f s" % (cores, times[cores], setup)),
            "one_core": {"value": n / times[1] / 1e6, "seconds": round(times[1], 2), "cores": 1},
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def profiled_traffic(kernel, precision):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when the kernel source has changed since the counters
    were taken (or the summary does not cover this precision)."""
    import hashlib
    if precision != "c64" or kernel != "k_translate_gemm":
        return None
    prof = os.path.join(ROOT, "profiles", "k_translate_gemm_sphere201720_c64.md")
    src = os.path.join(ROOT, "paper_1801_03589_amd", "csrc", "kernels.hip")
    try:
        text = open(prof).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    if ("sha256 prefix `%s`" % sha) not in text:
        return None
    for line in text.splitlines():
        if line.startswith("traffic_bytes_per_launch:"):
            return int(line.split(":")[1])
    return None


def dense_rows_error(nesa, torch, op, n, stream):
    """||(Z_NESA x)[rows] - (Z x)[rows]|| / ||(Z x)[rows]|| on the stored dense
    rows of the bench sphere (x = synth.complex_normal(n, 0); the rows and values
    come from the oracle alone, tests/golden/make_dense_rows.py)."""
    import synth
    path = os.path.join(ROOT, "tests", "golden", "dense_rows_sphere201720.json")
    with open(path) as f:
        g = json.load(f)
    if g["n"] != n:
        return None
    rows = np.array(g["rows"])
    yd = np.array(g["y_re"]) + 1j * np.array(g["y_im"])
    x = torch.from_numpy(synth.complex_normal(n, 0)).to(torch.complex64).cuda()
    y = torch.empty_like(x)
    nesa.matvec(op, x, y, stream=stream)
    torch.cuda.synchronize()
    yr = y.cpu().numpy().astype(np.complex128)[rows]
    return {"dense_rows": int(len(rows)), "rel_err": float(np.linalg.norm(yr - yd) / np.linalg.norm(yd))}


def split_section(args, nesa, torch, tree, near, far, n, stream, fp32_ms, fp32_batched_ms):
    """The bench sphere with split-bf16x3 translations and transfers: product
    time at one and at `nrhs` right-hand sides next to the complex64 (FP32
    matrix-core) times of the same operator, and the split product's error
    against the complex64 one; the same for the split with fp16 parts."""
    R = max(1, args.nrhs)
    ops = nesa.op_create(tree, near, far, nesa.C64_SPLIT, max_nrhs=R)
    x = torch.from_numpy(synth_rhs(n, 1)[0]).to(torch.complex64).cuda()
    y = torch.empty_like(x)
    X = torch.from_numpy(synth_rhs(n, R)).to(torch.complex64).cuda()
    Y = torch.empty_like(X)
    out = {}
    for name, xx, yy, rr, reps in (("1", x, y, 1, args.steps), (str(R), X, Y, R, max(3, args.steps // 4))):
        for _ in range(3):
            nesa.matvec(ops, xx, yy, rr, stream=stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            nesa.matvec(ops, xx, yy, rr, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        out["ms_per_product_nrhs" + name] = round(e0.elapsed_time(e1) / reps, 4)
    out["fp32_ms_per_product_nrhs1"] = round(fp32_ms, 4)
    if fp32_batched_ms is not None:
        out["fp32_ms_per_product_nrhs%d" % R] = round(fp32_batched_ms, 4)
    # error of the split product against the complex64 product (one right-hand side)
    op32 = nesa.op_create(tree, near, far, nesa.C64)
    y32 = torch.empty_like(x)
    nesa.matvec(op32, x, y32, stream=stream)
    nesa.matvec(ops, x, y, stream=stream)
    torch.cuda.synchronize()
    out["rel_diff_vs_complex64"] = float(torch.linalg.norm(y - y32) / torch.linalg.norm(y32))
    # the same products with fp16 parts (scaled operands, about 22 bits each)
    oph = nesa.op_create(tree, near, far, nesa.C64_SPLIT_FP16, max_nrhs=R)
    fp16 = {}
    for name, xx, yy, rr, reps in (("1", x, y, 1, args.steps), (str(R), X, Y, R, max(3, args.steps // 4))):
        for _ in range(3):
            nesa.matvec(oph, xx, yy, rr, stream=stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            nesa.matvec(oph, xx, yy, rr, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        fp16["ms_per_product_nrhs" + name] = round(e0.elapsed_time(e1) / reps, 4)
    nesa.matvec(oph, x, y, stream=stream)
    torch.cuda.synchronize()
    fp16["rel_diff_vs_complex64"] = float(torch.linalg.norm(y - y32) / torch.linalg.norm(y32))
    out["fp16_parts"] = fp16
    del oph, op32
    # the R incidences of the batched GMRES line solved in lock step with the
    # split operator and the near-list Schwarz preconditioner (set up on the
    # device), to 1e-4 (compare with gmres.batched.plain_fp32.one_at_a_time)
    B = torch.empty(R, n, dtype=torch.complex64, device="cuda")
    th = math.radians(30.0)
    for r in range(R):
        ph = 2.0 * math.pi * r / R
        k = [math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)]
        e = [math.cos(th) * math.cos(ph), math.cos(th) * math.sin(ph), -math.sin(th)]
        nesa.rhs_plane_wave(ops, k, e, B[r], stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nesa.precond_setup(ops, nesa.PRECOND_SCHWARZ)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    Xs = torch.zeros_like(B)
    t0 = time.perf_counter()
    rc, rep, _ = nesa.gmres_solve(ops, B, Xs, nrhs=R, restart=50, max_iters=args.gmres_iters, tol=1e-4,
                                  precond=nesa.PRECOND_SCHWARZ, stream=stream, check=False)
    torch.cuda.synchronize()
    out["schwarz_batched_solve"] = {"nrhs": R, "seconds": round(time.perf_counter() - t0, 3),
                                    "setup_s": round(setup_s, 3), "iters": [r_["iters"] for r_ in rep],
                                    "max_true_rel_residual": max(r_["true_rel_residual"] for r_ in rep),
                                    "converged": rc == 0}
    log("split + Schwarz batched GMRES: %.2f s" % out["schwarz_batched_solve"]["seconds"])
    del ops
    return out


def accurate_section(args, nesa, torch, tree, near, n, stream):
    """The bench sphere with d0 = 5 equivalent sources per box (Q = 576, 256,
    144, 81): the setting whose truncation error against the dense matrix is
    below 1e-3; product time and that error."""
    t0 = time.perf_counter()
    far5 = nesa.assemble_translations(tree, d0=5, tau=1e-8)
    op5 = nesa.op_create(tree, near, far5, nesa.C64)
    setup = time.perf_counter() - t0
    info = tree.info()
    Q = [int(q) for q in far5.q(info["L"] - info["l0"] + 1)]
    x = torch.from_numpy(np.ones(n, dtype=np.complex64)).cuda()
    y = torch.empty_like(x)
    for _ in range(5):
        nesa.matvec(op5, x, y, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        nesa.matvec(op5, x, y, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    out = {"d0": 5, "Q": Q, "ms_per_product": round(ms, 4),
           "Munknowns_matvec_per_s": round(n / (ms * 1e-3) / 1e6, 2), "setup_s": round(setup, 2),
           "truncation_error": dense_rows_error(nesa, torch, op5, n, stream)}
    del op5, far5
    return out


def gmres_section(args, nesa, torch, op, info, x, stream):
    """Time to a 1e-4 relative residual, GMRES(50) around the same operator:
    plain, with the near-list Schwarz preconditioner, and with the learned
    per-leaf network on top of it (trained here on pairs from the method's own
    Schwarz solves of other incidences; training time reported apart)."""
    import synth
    tol, restart = 1e-4, 50
    b = torch.empty_like(x)
    nesa.rhs_plane_wave(op, [0, 0, 1], [1, 0, 0], b, stream=stream)

    def solve(pc, max_iters):
        xs = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, rep, _ = nesa.gmres_solve(op, b, xs, restart=restart, max_iters=max_iters, tol=tol,
                                      precond=pc, stream=stream, check=False)
        torch.cuda.synchronize()
        r = rep[0]
        return {"iters": r["iters"], "seconds": round(time.perf_counter() - t0, 3),
                "true_rel_residual": r["true_rel_residual"], "converged": rc == 0,
                "fell_back": r["fell_back"]}

    out = {"tol": tol, "restart": restart, "rhs": "plane wave along +z, x-polarised"}
    out["plain_fp32"] = solve(nesa.PRECOND_NONE, args.gmres_iters)
    t0 = time.perf_counter()
    nesa.precond_setup(op, nesa.PRECOND_SCHWARZ)
    setup_s = time.perf_counter() - t0
    log("plain GMRES: %d iterations" % out["plain_fp32"]["iters"])
    out["schwarz_fp32"] = solve(nesa.PRECOND_SCHWARZ, args.gmres_iters)
    out["schwarz_fp32"]["setup_s"] = round(setup_s, 2)
    # training pairs: Schwarz solves of two other incidences
    t0 = time.perf_counter()
    Rs, Es = [], []
    for d, p in (([1.0, 0, 0], [0, 0, 1.0]), ([0, 0.6, 0.8], [1.0, 0, 0])):
        bt = torch.empty_like(b)
        nesa.rhs_plane_wave(op, d, p, bt, stream=stream)
        xt = torch.zeros_like(bt)
        _, rep, _ = nesa.gmres_solve(op, bt, xt, restart=restart, max_iters=600, tol=1e-6,
                                     precond=nesa.PRECOND_SCHWARZ, stream=stream, check=False)
        ks = sorted(set([0] + list(np.linspace(1, max(2, rep[0]["iters"] - 1), 6).astype(int))))
        R, E = nesa.solve_pairs(op, bt, xt, ks, restart=restart, precond=nesa.PRECOND_SCHWARZ)
        Rs.append(R)
        Es.append(E)
    S = 32 * int(math.ceil(info["max_leaf"] / 32))
    net = nesa.Mlp(op, S, 128, nesa.PRECOND_SCHWARZ, synth.mlp_weights(S, 128, seed=1))
    net.set_data(torch.cat(Rs), torch.cat(Es))
    hist = net.train(300, lr=1e-3)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    nesa.op_set_mlp(op, net)
    out["learned_fp32"] = solve(nesa.PRECOND_LEARNED, args.gmres_iters)
    out["learned_fp32"].update({"train_s": round(train_s, 2), "pairs": int(sum(r.shape[0] for r in Rs)),
                                "s_max": S, "hidden": 128, "loss_first": round(float(hist[0]), 4),
                                "loss_last": round(float(hist[-1]), 4)})
    nesa.op_set_mlp(op, None)
    out["max_iters"] = args.gmres_iters
    if args.nrhs > 1:
        out["batched"] = gmres_batched(args, nesa, torch, op, b, tol, restart, stream)
    return out


AIRCRAFT_SMALL = dict(fuselage_radius=0.8, fuselage_length=6.0, span=2.5, chord_root=1.5, chord_tip=0.6,
                      thickness=0.3, wing_x=2.5, gap=0.1)


def learned_family_section(args, nesa, torch, stream):
    """The learned preconditioner on the aircraft family: the network (one
    set of weights, carried from body to body) is trained on residual / error
    pairs of the method's own base-preconditioned FGMRES solves of bodies with
    seeds 100 .. 100 + n - 1 (about 48k unknowns each), then FGMRES(50) to 1e-4
    on the held-out body of seed 999: plain, block-diagonal, learned on
    block-diagonal, Schwarz, learned on Schwarz (two incidences each)."""
    import synth
    tol, restart, cap = 1e-4, 50, 1500
    incid = [([1.0, 0, 0], [0, 0, 1.0]), ([0, 0.6, 0.8], [1.0, 0, 0]), ([0, 0, 1.0], [0, 1.0, 0]),
             ([0.6, 0.8, 0], [0, 0, 1.0])]

    def build(seed):
        # the family: dimensions drawn from the seed around the small member
        rg = np.random.default_rng(seed)
        kw = dict(AIRCRAFT_SMALL)
        kw.update(fuselage_radius=float(rg.uniform(0.6, 0.9)), fuselage_length=float(rg.uniform(5.0, 8.0)),
                  span=float(rg.uniform(2.0, 3.2)), chord_root=float(rg.uniform(1.2, 1.8)))
        v, t = synth.aircraft_like(seed, **kw)
        tr = nesa.build_tree(v, t, 0.25)
        op = nesa.op_create(tr, nesa.assemble_near_device(tr), nesa.assemble_translations(tr, d0=3, tau=1e-8),
                            nesa.C64)
        nesa.precond_setup(op, nesa.PRECOND_SCHWARZ)
        return tr, op

    def rhs(op, n, d, p_):
        b = torch.empty(n, dtype=torch.complex64, device="cuda")
        nesa.rhs_plane_wave(op, d, p_, b, stream=stream)
        return b

    def solve(op, b, pc, max_iters=cap, tol_=tol):
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, rep, _ = nesa.gmres_solve(op, b, x, restart=restart, max_iters=max_iters, tol=tol_, precond=pc,
                                      stream=stream, check=False)
        torch.cuda.synchronize()
        return x, {"iters": rep[0]["iters"], "seconds": round(time.perf_counter() - t0, 3), "converged": rc == 0,
                   "true_rel_residual": rep[0]["true_rel_residual"], "fell_back": rep[0]["fell_back"]}

    S, H = 256, 128
    out = {"family": "synth.aircraft_like(seed) with fuselage radius U(0.6, 0.9), length U(5, 8), span U(2, 3.2), "
                     "root chord U(1.2, 1.8) drawn from the seed, wing thickness 0.3", "s_max": S,
           "hidden": H, "tol": tol, "restart": restart, "max_iters": cap}
    for base, bname in ((nesa.PRECOND_BLOCKDIAG, "blockdiag"), (nesa.PRECOND_SCHWARZ, "schwarz")):
        theta = synth.mlp_weights(S, H, seed=1)
        t0 = time.perf_counter()
        losses, npairs, sizes = [], 0, []
        for seed in range(100, 100 + args.learned_bodies):
            tr, op = build(seed)
            n = tr.info()["n_rwg"]
            sizes.append(n)
            Rs, Es = [], []
            for d, p_ in incid[:2]:
                b = rhs(op, n, d, p_)
                xs, _ = solve(op, b, nesa.PRECOND_SCHWARZ, 600, 1e-6)       # converged solution
                ks = [0, 2, 5, 10, 20, 40]
                R, E = nesa.solve_pairs(op, b, xs, ks, restart=restart, precond=base)
                Rs.append(R)
                Es.append(E)
            net = nesa.Mlp(op, S, H, base, theta)
            net.set_data(torch.cat(Rs), torch.cat(Es))
            hist = net.train(200, lr=1e-3)
            losses.append([round(float(hist[0]), 4), round(float(hist[-1]), 4)])
            theta = net.get_params()
            npairs += sum(r.shape[0] for r in Rs)
            del net, op, tr
        train_s = time.perf_counter() - t0
        tr, op = build(999)
        n = tr.info()["n_rwg"]
        net = nesa.Mlp(op, S, H, base, theta)
        nesa.op_set_mlp(op, net)
        res = {"train_bodies": len(sizes), "train_unknowns": [min(sizes), max(sizes)], "pairs": npairs,
               "train_s": round(train_s, 1), "loss_first_last_per_body": losses, "held_out_unknowns": n}
        for i, (d, p_) in enumerate(incid[2:]):
            b = rhs(op, n, d, p_)
            r = {}
            if bname == "blockdiag":
                _, r["plain"] = solve(op, b, nesa.PRECOND_NONE)
            _, r[bname] = solve(op, b, base)
            _, r["learned_" + bname] = solve(op, b, nesa.PRECOND_LEARNED)
            res["incidence_%d" % i] = r
        out[bname] = res
        log("learned on %s: %s" % (bname, {k: v for k, v in res.items() if k.startswith("incidence")}))
        nesa.op_set_mlp(op, None)
        del net, op, tr
    return out


def gmres_batched(args, nesa, torch, op, b, tol, restart, stream):
    """The batched form of the solve: nrhs incidences (wave vectors on a 30-degree
    cone, theta-polarised) in one lock-step GMRES (one multi-RHS product per
    iteration), plain and Schwarz-preconditioned, against the same incidences
    solved one at a time."""
    R = args.nrhs
    n = b.shape[0]
    B = torch.empty(R, n, dtype=b.dtype, device=b.device)
    th = math.radians(30.0)
    for r in range(R):
        ph = 2.0 * math.pi * r / R
        k = [math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)]
        e = [math.cos(th) * math.cos(ph), math.cos(th) * math.sin(ph), -math.sin(th)]
        nesa.rhs_plane_wave(op, k, e, B[r], stream=stream)

    def run(pc, batched):
        X = torch.zeros_like(B)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if batched:
            rc, rep, _ = nesa.gmres_solve(op, B, X, nrhs=R, restart=restart, max_iters=args.gmres_iters,
                                          tol=tol, precond=pc, stream=stream, check=False)
            ok = rc == 0
        else:
            rep, ok = [], True
            for r in range(R):
                x1 = torch.zeros_like(B[r])
                rc, rp, _ = nesa.gmres_solve(op, B[r].clone(), x1, restart=restart, max_iters=args.gmres_iters,
                                             tol=tol, precond=pc, stream=stream, check=False)
                rep += rp
                ok = ok and rc == 0
        torch.cuda.synchronize()
        return {"seconds": round(time.perf_counter() - t0, 3), "iters": [r["iters"] for r in rep],
                "max_true_rel_residual": max(r["true_rel_residual"] for r in rep), "converged": ok}

    out = {"nrhs": R, "incidences": "theta = 30 deg, phi = 360 r / nrhs deg, theta-polarised"}
    for name, pc in (("plain_fp32", nesa.PRECOND_NONE), ("schwarz_fp32", nesa.PRECOND_SCHWARZ)):
        out[name] = {"batched": run(pc, True)}
        log("batched GMRES (%s): %.2f s" % (name, out[name]["batched"]["seconds"]))
        out[name]["one_at_a_time"] = run(pc, False)
        log("sequential GMRES (%s): %.2f s" % (name, out[name]["one_at_a_time"]["seconds"]))
    return out


def batched_section(args, nesa, torch, tree, near, far, prec, dt, n, stream):
    """Several right-hand sides in one product (channels = 4 x nrhs through
    the GEMM tiles): Munknowns * matvec / s counted over all right-hand sides."""
    if args.nrhs <= 1:
        return None
    opb = nesa.op_create(tree, near, far, prec, max_nrhs=args.nrhs)
    X = torch.from_numpy(synth_rhs(n, args.nrhs)).to(dt).cuda()
    Y = torch.empty_like(X)
    for _ in range(2):
        nesa.matvec(opb, X, Y, args.nrhs, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = max(3, args.steps // 4)
    e0.record(stream)
    for _ in range(reps):
        nesa.matvec(opb, X, Y, args.nrhs, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"nrhs": args.nrhs, "ms_per_product": round(ms, 4),
            "Munknowns_matvec_per_s": round(n * args.nrhs / (ms * 1e-3) / 1e6, 2)}


def schwarz_section(args, nesa, torch):
    """Device setup of the near-list Schwarz preconditioner of the bench sphere
    (complex64, one right-hand side): per leaf a, the LU of the W_a x W_a
    near-list matrix and S_a unit solves.  Algorithmic work: 8/3 W^3 real flops
    per LU plus 8 W^2 S per leaf for the solves (complex FMA = 8 flops)."""
    import synth
    v, t = synth.icosphere(args.nu, args.radius)
    tree = nesa.build_tree(v, t, 0.25)
    near = nesa.assemble_near_device(tree)
    far = nesa.assemble_translations(tree, d0=3, tau=1e-8)
    S, W = tree.leaf_sizes()
    flops = float(np.sum(8.0 / 3.0 * W.astype(float) ** 3 + 8.0 * W.astype(float) ** 2 * S))
    runs = []
    for _ in range(2):
        op = nesa.op_create(tree, near, far, nesa.C64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nesa.precond_setup(op, nesa.PRECOND_SCHWARZ)
        torch.cuda.synchronize()
        runs.append(time.perf_counter() - t0)
        del op
    best = min(runs)
    log("Schwarz setup on the device: %.3f s (%d leaves, W mean %.0f, max %d)" % (best, len(W), W.mean(), W.max()))
    return {"leaves": int(len(W)), "W_mean": round(float(W.mean()), 1), "W_max": int(W.max()),
            "setup_s": [round(x, 4) for x in runs], "algorithmic_tflop": round(flops / 1e12, 3),
            "achieved_tflops": round(flops / best / 1e12, 2), "fp32_peak_frac": round(flops / best / PEAK_FP32, 4)}


def aircraft_section(args, nesa, torch, stream):
    """Aircraft-like body (seed 3: 959,364 unknowns, 50-wavelength fuselage, two
    swept wings), leaf 0.25, far field from the 4-wavelength level (l0 = 4:
    Q = 1156, 441, 196, 81, 49), 64 plane-wave incidences in one batched
    product with split-bf16x3 translations and transfers (FP32 accumulation).
    Munknowns * matvec / s counted over all right-hand sides; the translation
    stage's roofline against the bf16 matrix-core peak (the dtype its products
    run in), its algorithmic flops 8 x 4 nrhs x Q^2 per pair."""
    import synth
    R = args.aircraft_nrhs
    if R <= 0:
        return None
    setup = {}
    t0 = time.perf_counter()
    v, t = synth.aircraft_like(3)
    tree = nesa.build_tree(v, t, 0.25, l0_max=4)
    info = tree.info()
    setup["tree_s"] = time.perf_counter() - t0
    log("aircraft: tree of %d unknowns, levels %d..%d" % (info["n_rwg"], info["l0"], info["L"]))
    t0 = time.perf_counter()
    near = nesa.assemble_near_device(tree)
    setup["near_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    far = nesa.assemble_translations(tree, d0=3, tau=1e-8)
    setup["far_s"] = time.perf_counter() - t0
    nl = info["L"] - info["l0"] + 1
    Q = [int(q) for q in far.q(nl)]
    log("aircraft: far-field operators (Q %s)" % Q)
    out = {"workload": "aircraft_like_seed3_%drwg" % info["n_rwg"], "n_unknowns": info["n_rwg"], "nrhs": R,
           "leaf_lambda": 0.25, "levels": [info["l0"], info["L"]], "Q": Q, "boxes": info["n_box"],
           "pairs": info["n_pairs"], "near_entries": info["near_entries"]}
    n = info["n_rwg"]
    precs = [("split", nesa.C64_SPLIT)] + ([("c64", nesa.C64)] if args.aircraft_fp32 else [])
    for name, prec in precs:
        t0 = time.perf_counter()
        op = nesa.op_create(tree, near, far, prec, max_nrhs=R)
        setup["op_%s_s" % name] = time.perf_counter() - t0
        X = torch.from_numpy(synth.complex_normal((R, n), 5)).to(torch.complex64).cuda()
        Y = torch.empty_like(X)
        t0 = time.perf_counter()
        nesa.matvec(op, X, Y, R, stream=stream)          # first product: tile tuning
        torch.cuda.synchronize()
        setup["first_product_%s_s" % name] = time.perf_counter() - t0
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = 3
        e0.record(stream)
        for _ in range(reps):
            nesa.matvec(op, X, Y, R, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        lt = nesa.matvec_launch_times(op, X, Y, stream=stream, nrhs=R)
        kern = {}
        for kind, lev, m in lt:
            e = kern.setdefault(kind, {"ms": 0.0, "launches": 0, "flops": 0.0})
            e["ms"] += m
            e["launches"] += 1
            i = lev - info["l0"]
            if kind == "translate_gemm":
                e["flops"] += 8 * 4 * R * info["n_pairs"][i] * Q[i] * Q[i]
            elif kind in ("upward_gemm", "downward_gemm"):
                e["flops"] += info["n_box"][i] * 8 * 4 * R * Q[i - 1] * Q[i]
        tr_ = kern.get("translate_gemm")
        peak = PEAK_BF16 if prec == nesa.C64_SPLIT else PEAK_FP32
        sec = {"ms_per_product": round(ms, 3),
               "Munknowns_matvec_per_s": round(n * R / (ms * 1e-3) / 1e6, 1),
               "launches": [[kind, lev, round(m, 3)] for kind, lev, m in lt],
               "kernels": {k: {"ms_per_product": round(v_["ms"], 3), "launches": v_["launches"],
                               "TFLOP/s": round(v_["flops"] / (v_["ms"] * 1e-3) / 1e12, 1) if v_["flops"] else None}
                           for k, v_ in kern.items()}}
        if tr_:
            ach = tr_["flops"] / (tr_["ms"] * 1e-3)
            sec["translate_roofline"] = {"bound": "mfma", "achieved": round(ach / 1e12, 1),
                                         "peak": peak / 1e12, "unit": "TFLOP/s", "frac": round(ach / peak, 4),
                                         "kernel": "k_translate_tm_split2" if prec == nesa.C64_SPLIT
                                         else "k_translate_tm"}
        out[name] = sec
        log("aircraft %s: %d right-hand sides, %.2f ms per product" % (name, R, ms))
        del op, X, Y
        torch.cuda.empty_cache()
    out["setup_s"] = {k: round(v_, 2) for k, v_ in setup.items()}
    return out


# The paper's own timed workload (2D model problem, N = 100 000, real FP64):
# best complete-product times it prints, with their hardware (context only)
PAPER_2D = {(50, 10): (100.0, "64 Xeon E5-4650 cores, SuperGlue"),
            (300, 100): (127.0, "64 Xeon E5-4650 cores, SuperGlue"),
            (400, 100): (None, "no complete-product time printed")}


def model2d_section(args, nesa, torch, stream):
    """The 2D potential problem at the paper's size and (P, Q) settings: one NESA
    product per step (near field + five far-field stages), charges resident on
    the GPU; the seeded curve stands in for the paper's (unpublished) one."""
    import synth
    n = 100000
    xy = synth.smooth_curve(n, 23)
    q = torch.from_numpy(synth.real_normal(n, 24)).cuda()
    phi = torch.empty_like(q)
    out = []
    for P, Q in ((50, 10), (300, 100), (400, 100)):
        t0 = time.perf_counter()
        op = nesa.Model2D(xy, P, Q)
        build = time.perf_counter() - t0
        info = op.info()
        for _ in range(5):
            op.matvec(q, phi, stream=stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            op.matvec(q, phi, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        paper_ms, hw = PAPER_2D[(P, Q)]
        out.append({"P": P, "Q": Q, "levels": [info["l0"], info["L"]], "boxes": info["n_box"],
                    "near_pairs": info["near_pairs"], "ms_per_product": round(ms, 4),
                    "Munknowns_per_s": round(n / (ms * 1e-3) / 1e6, 2),
                    "near_Gpairs_per_s": round(info["near_pairs"] / (ms * 1e-3) / 1e9, 1),
                    "build_s": round(build, 2), "paper_best_ms": paper_ms, "paper_hardware": hw})
        log("2D model P %d Q %d: %.4f ms per product" % (P, Q, ms))
        del op
    return {"n": n, "dtype": "f64", "runs": out}


def bodies_section(args, nesa, torch, prec, dt, stream):
    """A batch of uneven seeded bodies (spheroids, boxes, capped cylinders with
    2k to 50k unknowns, log-uniform) in one forest operator: every stage is one
    launch for all bodies; `nrhs` incidences per body.  Munknowns * matvec / s
    counted over all bodies and right-hand sides."""
    import synth
    if args.bodies <= 0:
        return None
    t0 = time.perf_counter()
    parts = {}
    bodies = synth.body_family(args.bodies, seed=4)
    parts["meshes_s"] = time.perf_counter() - t0
    tree = nesa.build_forest([(v, t) for v, t, _ in bodies], 0.25)
    parts["forest_s"] = time.perf_counter() - t0 - sum(parts.values())
    log("bodies: forest of %d unknowns built" % tree.info()["n_rwg"])
    near = nesa.assemble_near_device(tree)      # near-field blocks assembled on the GPU
    parts["near_s"] = time.perf_counter() - t0 - sum(parts.values())
    log("bodies: near field assembled")
    far = nesa.assemble_translations(tree, d0=3, tau=1e-8)
    parts["far_s"] = time.perf_counter() - t0 - sum(parts.values())
    log("bodies: far-field operators assembled")
    R = max(1, args.nrhs)
    op = nesa.op_create(tree, near, far, prec, max_nrhs=R)
    del near, far
    parts["op_s"] = time.perf_counter() - t0 - sum(parts.values())
    log("bodies: operator on the GPU")
    setup = time.perf_counter() - t0
    info = tree.info()
    n = info["n_rwg"]
    X = torch.from_numpy(synth.complex_normal((R, n), 2)).to(dt).cuda()
    Y = torch.empty_like(X)
    for _ in range(2):
        nesa.matvec(op, X, Y, R, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = max(3, args.steps // 4)
    e0.record(stream)
    for _ in range(reps):
        nesa.matvec(op, X, Y, R, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    sizes = [len(t) * 3 // 2 for _, t, _ in bodies]
    return {"bodies": args.bodies, "nrhs": R, "n_unknowns": n, "min_body": min(sizes), "max_body": max(sizes),
            "levels": [info["l0"], info["L"]], "ms_per_product": round(ms, 4),
            "Munknowns_matvec_per_s": round(n * R / (ms * 1e-3) / 1e6, 2), "setup_s": round(setup, 1),
            "setup_parts_s": {k: round(v, 2) for k, v in parts.items()}}


def synth_rhs(n, nrhs):
    import synth
    return synth.complex_normal((nrhs, n), 1)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: there is no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    from paper_1801_03589_amd import nesa

    if args.only_model2d:
        print(json.dumps({"model2d": model2d_section(args, nesa, torch, torch.cuda.current_stream())}))
        return
    if args.only_aircraft:
        print(json.dumps({"aircraft": aircraft_section(args, nesa, torch, torch.cuda.current_stream())}))
        return
    if args.only_schwarz:
        print(json.dumps({"schwarz_setup": schwarz_section(args, nesa, torch)}))
        return
    if args.only_learned_family:
        print(json.dumps({"learned_family": learned_family_section(args, nesa, torch, torch.cuda.current_stream())}))
        return
    prec = {"c64": nesa.C64, "c128": nesa.C128, "split": nesa.C64_SPLIT,
            "split_fp16": nesa.C64_SPLIT_FP16}[args.precision]
    esize = 16 if prec == nesa.C128 else 8
    dt = torch.complex128 if prec == nesa.C128 else torch.complex64
    setup = {}
    t0 = time.perf_counter()
    v, t = synth.icosphere(args.nu, args.radius)
    tree = nesa.build_tree(v, t, 0.25)
    info = tree.info()
    setup["tree_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    near = nesa.assemble_near_device(tree)      # near-field blocks assembled on the GPU
    setup["near_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    far = nesa.assemble_translations(tree, d0=3, tau=1e-8)
    setup["far_s"] = time.perf_counter() - t0
    nl = info["L"] - info["l0"] + 1
    Q = [int(q) for q in far.q(nl)]
    t0 = time.perf_counter()
    op = nesa.op_create(tree, near, far, prec, max_nrhs=max(1, args.nrhs))
    setup["upload_s"] = time.perf_counter() - t0
    n = info["n_rwg"]
    x = torch.from_numpy(synth.complex_normal(n, 0)).to(dt).cuda()
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    if args.counters:
        # counter passes: five products, then a plain copy of known size whose
        # FETCH_SIZE / WRITE_SIZE calibrate the counters (512 MiB read, 512 MiB written)
        for _ in range(5):
            nesa.matvec(op, x, y, stream=stream)
        torch.cuda.synchronize()
        log("products done")
        big = torch.ones(64 * 2 ** 20, dtype=torch.complex64, device="cuda")
        big2 = torch.empty_like(big)
        big2.copy_(big)
        torch.cuda.synchronize()
        log("copy of 512 MiB done")
        return
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
    # five further blocks of the same length: median (spread of the timing)
    blocks = []
    for _ in range(5):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            nesa.matvec(op, x, y, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        blocks.append(e0.elapsed_time(e1) / args.steps)
    repeat_ms = sorted(blocks)
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
        elif kind == "receive":
            e["bytes"] += alg["receive"]["bytes"]
            e["flops"] += alg["receive"]["flops"]
        elif kind in ("translate_sum",):
            # level -1: one launch for the sums of every level
            lv_range = range(len(Q)) if lev < 0 else [i]
            e["bytes"] += sum(2 * info["n_pairs"][j] * 4 * Q[j] * esize for j in lv_range)
        elif kind in ("upward_sum",):
            e["bytes"] += 2 * info["n_box"][i] * 4 * Q[i - 1] * esize
    dom = max(kern, key=lambda k: kern[k]["ms"])
    kd = kern[dom]
    sec = kd["ms"] * 1e-3
    if kd["bytes"] == 0 or dom.endswith("gemm") or dom.endswith("fp64"):
        # (split products: 16-bit matrix cores; their flops counted as complex
        # FP32 products, the x3 form issues three times as many)
        peak = 78.6e12 if prec == nesa.C128 else (PEAK_BF16 if prec in (nesa.C64_SPLIT, nesa.C64_SPLIT_FP16)
                                                  else PEAK_FP32)
        roof = {"bound": "mfma", "achieved": kd["flops"] / sec / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": kd["bytes"] / sec / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    split_prec = prec in (nesa.C64_SPLIT, nesa.C64_SPLIT_FP16)
    roof["kernel"] = {"translate_gemm": "k_translate_gemm_bf16x3 / k_gemm_om_split2" if split_prec
                      else "k_translate_gemm", "near_recv": "k_near_half",
                      "upward_gemm": "k_transfer_gemm", "downward_gemm": "k_transfer_gemm"}.get(dom, dom)
    roof["traffic"] = profiled_traffic(roof["kernel"], args.precision)
    roof["launches_per_product"] = kd["launches"]
    roof["avg_launch_ms"] = kd["ms"] / kd["launches"]
    kernels = {k: {"ms_per_product": round(v_["ms"], 4), "launches": v_["launches"],
                   "TFLOP/s": round(v_["flops"] / (v_["ms"] * 1e-3) / 1e12, 2) if v_["flops"] else None,
                   "GB/s": round(v_["bytes"] / (v_["ms"] * 1e-3) / 1e9, 1) if v_["bytes"] else None}
               for k, v_ in kern.items()}
    # whole-product roofline: sum over stages of max(bytes / HBM peak, flops / FP32 peak)
    peak_f = PEAK_FP32 if prec != nesa.C128 else 78.6e12
    t_roof = sum(max(alg[k]["bytes"] / PEAK_HBM, alg[k]["flops"] / peak_f)
                 for k in ("near_recv", "radiate", "upward", "downward", "translate"))
    phases = {}
    for k in names:
        s_ = phase_ms[k] * 1e-3
        phases[k] = {"ms": phase_ms[k], "GB/s": round(alg[k]["bytes"] / s_ / 1e9, 1),
                     "TFLOP/s": round(alg[k]["flops"] / s_ / 1e12, 2)}
    log("product: %.4f ms (%.1f Munknowns/s)" % (ms, value))
    gm = batched = bodies = model2d = accurate = aircraft = trunc = split = None
    if not args.only_product:
        trunc = dense_rows_error(nesa, torch, op, n, stream)
        trunc["bound"] = 3e-3
        log("truncation error on the dense rows: %.3e" % trunc["rel_err"])
        accurate = accurate_section(args, nesa, torch, tree, near, n, stream)
        log("d0 = 5: %.4f ms per product" % accurate["ms_per_product"])
        gm = gmres_section(args, nesa, torch, op, info, x, stream)
        log("GMRES done; batched right-hand sides")
        batched = batched_section(args, nesa, torch, tree, near, far, prec, dt, n, stream)
        log("split precision on the bench sphere")
        split = split_section(args, nesa, torch, tree, near, far, n, stream, ms,
                              batched["ms_per_product"] if batched else None) if prec == nesa.C64 else None
        del op
        log("batch of %d bodies" % args.bodies)
        bodies = bodies_section(args, nesa, torch, prec, dt, stream)
        log("2D model problem")
        model2d = model2d_section(args, nesa, torch, stream)
        aircraft = aircraft_section(args, nesa, torch, stream)
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
        "dtype": {"c64": "complex64", "c128": "complex128", "split": "complex64+bf16x3",
                  "split_fp16": "complex64+fp16x3"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "pec_sphere_r%gl_icosphere%d_%drwg" % (args.radius, args.nu, n),
                   "n_unknowns": n, "nrhs": 1, "leaf_lambda": 0.25, "levels": [info["l0"], info["L"]],
                   "Q": Q, "boxes": info["n_box"], "pairs": info["n_pairs"],
                   "near_entries": info["near_entries"], "near_entries_half": info["near_entries_half"],
                   "parallelism": "single_gpu"},
        "roofline": roof,
        "product_roofline": {"t_roof_ms": round(t_roof * 1e3, 4), "frac": round(t_roof * 1e3 / ms, 4),
                             "definition": "sum over stages of max(algorithmic bytes / 8 TB/s, "
                                           "algorithmic flops / matrix-core peak)"},
        "repeat_ms_per_step": {"median": round(repeat_ms[2], 4), "min": round(repeat_ms[0], 4),
                               "max": round(repeat_ms[4], 4), "blocks": 5},
        "phases": phases,
        "kernels": kernels,
        "launches": [[k, lev, round(m, 4)] for k, lev, m in launches],
        "wall_s_timed": round(wall, 4),
        "setup_s": {k: round(v_, 2) for k, v_ in setup.items()},
        "truncation_error": trunc,
        "accurate": accurate,
        "gmres": gm,
        "batched": batched,
        "split": split,
        "bodies": bodies,
        "model2d": model2d,
        "aircraft": aircraft,
    }
    if not args.no_cpu_baseline and not args.only_product:
        log("CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(v, t)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
