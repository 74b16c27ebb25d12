"""Benchmark of the LapH perambulator path on one MI355X.

A step is one perambulator for one source time: 4 * nev spin-diluted LapH
sources solved by the batched mixed-precision (FP16-with-norm inner, FP64
reliable updates) even-odd BiCGStab to a full-lattice residual of 1e-10, then
projected with the FP64 matrix-core GEMM onto the LapH vectors of every sink
timeslice.  The default workload is the 32^3 x 64 headline case (nev = 64,
256 RHS per source time, source times 0, 16, 32, 48 in turn); inputs are
seeded synthetic fields already resident in HBM when the timed region starts.

Prints one JSON line.  Only one GPU: ``--gpus N`` with N > 1 exits.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import laph_synth as ls  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6
# FP32 vector peak without packed-FP32 instructions (the build disables them):
# 256 CUs x 64 lanes x 2 flop (FMA) x 2.4 GHz
ALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
# flops per output site and RHS of a fused stage: 8 hops x 180 (projection 24,
# two SU(3) x colour-vector products 132, spin reconstruction 24) + two Hermitian
# 6x6 clover blocks 2 x 252
STAGE_FLOPS_PER_SITE_RHS = 8 * 180 + 2 * 252


def stage_bytes_per_site(prec, n_rhs, stage):
    """Algorithmic HBM bytes per output site of one launch of a fused stage.

    Each input spinor, output spinor (and, stage 2, the xpay input p and the
    shadow residual r^ of the fused <r^, v>) is moved once per RHS; the links
    (8 per output site) and the clover inverse of the output site once per launch."""
    sp = {"f64": 192, "f32": 96, "f16n": 52}[prec]
    link = {"f64": 144, "f32": 48, "f16n": 24}[prec]
    clov = {"f64": 576, "f32": 288, "f16n": 288}[prec]
    per_rhs = sp * (2 if stage == 1 else 4)
    return n_rhs * per_rhs + 8 * link + clov


def cpu_baseline(cfg, dims, U, v_src, seconds_budget=20.0):
    """The FP64 oracle timed on the host: full-lattice BiCGStab iterations on the
    headline lattice for one LapH source, scaled to RHS/s with the iteration count
    the oracle needs for 1e-10 on the same parameters (measured on 8^3 x 16).

    One iteration costs T(2 iterations) - T(1 iteration) of the oracle's solver
    (each call also forms the initial and the final true residual)."""
    from oracle import dirac, laph as olaph, solvers
    m0, csw = cfg["masses"][0], cfg["csw"]
    # iteration count at the same mass and gauge parameters on a small lattice
    small = (8, 8, 8, 16)
    Us = ls.gauge_field(small, cfg["seed_u"])
    Vs = ls.orthonormal_laph_vectors(small, 1, cfg["seed_v"])
    Ds = dirac.WilsonClover(Us, m0, csw)
    _, info = solvers.bicgstab(Ds.apply, olaph.laph_sources(Vs, 0)[:1], tol=1e-10)
    n_it = int(info["iters"][0])
    # full-size iterations on the bench's gauge field and first LapH vector, bounded
    D = dirac.WilsonClover(U, m0, csw)
    b = olaph.laph_sources(v_src, 0)[:1]
    D.apply(b)  # first touch

    def run(k_iters):
        t = time.perf_counter()
        solvers.bicgstab(D.apply, b, tol=1e-30, maxiter=k_iters, max_restarts=0)
        return time.perf_counter() - t

    t1, t2, reps = [], [], 0
    t_start = time.perf_counter()
    while reps < 4:
        t1.append(run(1))
        t2.append(run(2))
        reps += 1
        if time.perf_counter() - t_start > seconds_budget:
            break
    per_iter = max(min(t2) - min(t1), 1e-9)
    rhs_per_s = 1.0 / (per_iter * n_it)
    cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    return {"value": rhs_per_s, "unit": "RHS/s", "cores": cores, "kind": "oracle",
            "sample": "1 LapH source on %s: the FP64 oracle BiCGStab run for 1 and for 2 iterations (%d times "
                      "each); one iteration = the difference of the fastest runs (%.2f s), times the %d "
                      "iterations the oracle needs for 1e-10 at m0=%g (measured on 8^3x16)"
                      % ("x".join(map(str, dims)), reps, per_iter, n_it, m0)}


# The stencil sources whose counters a stored traffic figure describes.
STAGE_SOURCES = ["dslash_kernels.h", "dslash_lds.h", "laph_internal.h", "dslash_f16.hip", "dslash_f32.hip",
                 "dslash_f64.hip", "dslash.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stage1_pmc_traffic.md")


def stage_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in STAGE_SOURCES:
        with open(os.path.join(ROOT, "paper_2510_26313_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(key):
    """HBM bytes per launch of the dominant stage from the committed counter
    summary, or None when there is none for this shape or the stencil sources
    changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    digest = stage_source_digest()
    for ln in lines:
        if ln.startswith("traffic:"):
            f = dict(kv.split("=", 1) for kv in ln[len("traffic:"):].split())
            if f.get("key") == key and f.get("sources") == digest:
                return float(f["bytes_per_launch"])
    return None


def progress(msg):
    """A progress line on stderr (stdout carries only the result line)."""
    print("[bench] %s" % msg, file=sys.stderr, flush=True)


def _timed(torch, fn):
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return r, time.perf_counter() - t


def _solve_summary(st, n, dt):
    return {"rhs_per_s": round(n / dt, 2), "mean_iters": round(float(np.mean([s["iters"] for s in st])), 2),
            "mean_updates": round(float(np.mean([s["updates"] for s in st])), 2),
            "max_true_res": max(s["true_res"] for s in st)}


def extra_suite(laph, torch):
    """Secondary measurements of the other workloads (outside the timed region):
    16^3x32 single-RHS solves per inner precision, the 24^3x48 four-mass batched
    solve against the plain FP64 single-RHS solver, the forward / backward times of
    the differentiable perambulator at 16^3x32, and the LapH vectors (64 lowest
    eigenpairs of -Delta per timeslice) at 32^3x64."""
    out = {}
    tol = 1e-10
    # 16^3 x 32: 128 RHS at t0 = 0, one RHS after another
    cfg = ls.CONFIGS["single_rhs_16x16x16x32"]
    dims = cfg["dims"]
    lat = laph.Lattice(dims)
    lat.load_gauge(torch.from_numpy(ls.gauge_field(dims, cfg["seed_u"])).cuda())
    lat.set_masses([cfg["masses"][0]], cfg["csw"])
    Vd = torch.from_numpy(ls.orthonormal_laph_vectors(dims, cfg["nev"], cfg["seed_v"])).cuda()
    B = lat.make_sources(Vd, 0)
    single = {}
    for prec in ("f64", "f32", "f16n"):
        p = laph.default_params(inner_prec=prec, batched=0, rhs_tile=1, stencil=1, traversal=1)
        lat.solve_raw(B[:2].contiguous(), 0, tol, p)
        (_, st), dt = _timed(torch, lambda: lat.solve_raw(B, 0, tol, p))
        single["single_rhs_" + prec] = _solve_summary(st, B.shape[0], dt)
    tuned = lat.autotune("f16n", B.shape[0], 0)
    lat.autotune("f64", B.shape[0], 0)   # the reliable-update stages' shape, outside the timing
    p = laph.default_params(inner_prec="f16n", stencil=tuned["stencil"], rhs_tile=tuned["rhs_tile"],
                            traversal=tuned["traversal"])
    (_, st), dt = _timed(torch, lambda: lat.solve_raw(B, 0, tol, p))
    single["batched_f16n"] = _solve_summary(st, B.shape[0], dt)
    out["16x16x16x32_128rhs_m0.05"] = single
    del lat, Vd, B
    torch.cuda.empty_cache()

    # 24^3 x 48: 256 RHS over four masses in one batched solve
    cfg = ls.CONFIGS["multimass_24x24x24x48"]
    dims = cfg["dims"]
    lat = laph.Lattice(dims)
    lat.load_gauge(torch.from_numpy(ls.gauge_field(dims, cfg["seed_u"])).cuda())
    lat.set_masses(list(cfg["masses"]), cfg["csw"])
    Vd = torch.from_numpy(ls.orthonormal_laph_vectors(dims, cfg["nev"], cfg["seed_v"])).cuda()
    B = lat.make_sources(Vd, 0)
    mi = ls.rhs_masses(cfg)
    tuned = lat.autotune("f16n", B.shape[0], 0)
    lat.autotune("f64", B.shape[0], 0)
    p = laph.default_params(inner_prec="f16n", stencil=tuned["stencil"], rhs_tile=tuned["rhs_tile"],
                            traversal=tuned["traversal"])
    (X, st), dt = _timed(torch, lambda: lat.solve_raw(B, mi, tol, p))
    del X
    multi = {"batched_f16n": _solve_summary(st, B.shape[0], dt), "tuned": tuned, "per_mass": {}}
    for m, m0 in enumerate(cfg["masses"]):
        it = [s["iters"] for s, mm in zip(st, mi) if mm == m]
        multi["per_mass"]["%g" % m0] = {"rhs": len(it), "iters_min": min(it), "iters_max": max(it)}
    pick = [0, 39, 40, 111, 112, 175, 176, 255]   # two per mass
    Bs = B[pick].contiguous()
    p64 = laph.default_params(inner_prec="f64", batched=0, rhs_tile=1, stencil=1, traversal=1)
    (_, st64), dt64 = _timed(torch, lambda: lat.solve_raw(Bs, [mi[r] for r in pick], tol, p64))
    multi["single_rhs_f64_sample"] = _solve_summary(st64, len(pick), dt64)
    multi["speedup_of_batched_mixed"] = round(multi["batched_f16n"]["rhs_per_s"] / multi["single_rhs_f64_sample"]["rhs_per_s"], 2)
    out["24x24x24x48_256rhs_4masses"] = multi
    del lat, Vd, B, Bs
    torch.cuda.empty_cache()

    # 16^3 x 32: differentiable perambulator, L = sum |tau[t = 8]|^2, FP32 inner
    cfg = ls.CONFIGS["gradients_8x8x8x8"]
    dims = cfg["dims_timing"]
    lat = laph.Lattice(dims)
    lat.load_gauge(torch.from_numpy(ls.gauge_field(dims, cfg["seed_u"])).cuda())
    lat.csw = cfg["csw"]
    Vd = torch.from_numpy(ls.orthonormal_laph_vectors(dims, cfg["nev"], cfg["seed_v"])).cuda()
    grad = {}
    for rep in range(2):   # the first pass warms up
        B = lat.make_sources(Vd, 0).requires_grad_(True)
        m0 = torch.tensor(cfg["masses"][0], dtype=torch.float64, requires_grad=True)
        tau, tf = _timed(torch, lambda: laph.project(lat, laph.solve(lat, B, m0, tol, inner_prec="f32"), Vd))
        L = (tau[cfg["t_sink_timing"]].abs() ** 2).sum()
        _, tb = _timed(torch, lambda: L.backward())
        grad = {"rhs": int(B.shape[0]), "forward_s": round(tf, 4), "backward_s": round(tb, 4),
                "backward_over_forward": round(tb / tf, 3), "grad_m0": float(m0.grad)}
    out["16x16x16x32_gradients"] = grad
    del lat, Vd
    torch.cuda.empty_cache()

    out["32x32x32x64_laph_vectors_nev64"] = laph_vectors_run(laph, torch)
    out["32x32x32x64_contractions_nev64"] = contractions_run(laph, torch)
    return out


def laph_vectors_run(laph, torch):
    """The 64 lowest eigenpairs of -Delta on all 64 timeslices of 32^3 x 64 (the LapH
    vectors), and the Laplacian stencil's rate on 8 vectors per timeslice."""
    cfg = ls.CONFIGS["perambulator_32x32x32x64"]
    dims = cfg["dims"]
    lat = laph.Lattice(dims)
    lat.load_gauge(torch.from_numpy(ls.gauge_field(dims, cfg["seed_u"])).cuda())
    (V, lam, info), dt = _timed(torch, lambda: lat.laplacian_eigvecs(cfg["nev"], tol=1e-10))
    X = V[:, :8].contiguous()
    lat.apply_laplacian(X)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        lat.apply_laplacian(X)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    vs = dims[0] * dims[1] * dims[2]
    # algorithmic bytes per site: in + out of every vector (96 B each) + the three
    # links of the site (432 B, read once for all vectors)
    gb = (8 * 96 + 432) * vs * dims[3] / (ms * 1e-3) / 1e9
    res = {"seconds": round(dt, 3), "iterations": info["iters"], "max_residual": info["residual"],
           "lowest_eigenvalue": float(lam.min()), "largest_returned_eigenvalue": float(lam.max()),
           "laplacian_8vec_ms": round(ms, 4), "laplacian_8vec_gbs": round(gb, 1),
           "laplacian_8vec_hbm_frac": round(gb / HBM_PEAK_GBS, 4)}
    del lat, V, X
    torch.cuda.empty_cache()
    return res


def contractions_run(laph, torch, n_mom=4, reps=3):
    """Meson doublets and baryon triplets of 64 LapH vectors on every timeslice of
    32^3 x 64 for n_mom momenta: average time per call (HIP events over reps calls
    after one warm call) and the rates against the FP64 matrix-core and HBM peaks."""
    cfg = ls.CONFIGS["perambulator_32x32x32x64"]
    dims, nev = cfg["dims"], cfg["nev"]
    lat = laph.Lattice(dims)
    Vd = torch.from_numpy(ls.orthonormal_laph_vectors(dims, nev, cfg["seed_v"])).cuda()
    moms = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0), (0, 0, 1), (1, 0, 1), (0, 1, 1), (1, 1, 1)][:n_mom]
    vs = dims[0] * dims[1] * dims[2]
    out = {"momenta": n_mom}
    for name, fn in (("doublets", lat.meson_doublets), ("triplets", lat.baryon_triplets)):
        r = fn(Vd, moms)
        del r
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            r = fn(Vd, moms)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out_bytes = r.numel() * 16
        del r
        v_bytes = Vd.numel() * 16
        if name == "doublets":
            # complex multiply-adds: nev^2 entries x 3 vs terms per (t, p)
            flops = 8.0 * nev * nev * 3 * vs * dims[3] * n_mom
        else:
            # the distinct triplets l < m < n, 3 vs terms each
            flops = 8.0 * (nev * (nev - 1) * (nev - 2) // 6) * 3 * vs * dims[3] * n_mom
        out[name] = {"ms": round(ms, 3), "tflops": round(flops / (ms * 1e-3) / 1e12, 3),
                     "fp64_mfma_frac": round(flops / (ms * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS, 4),
                     "gbs_v_once_plus_output": round((v_bytes + out_bytes) / (ms * 1e-3) / 1e9, 1)}
    del lat, Vd
    torch.cuda.empty_cache()
    return out


def stage_key(args, dims):
    return "%s/%s/n%d/s%d/t%d/v%d" % ("x".join(map(str, dims)), args.prec, args.chunk, args.stencil,
                                      args.rhs_tile, args.traversal)


def pmc_probe(args, cfg, torch, laph):
    """Launch the dominant stage of the bench workload (shape given on the command
    line; unit gauge, the traffic does not depend on the values) and a plain
    copy of known size, for hardware-counter runs."""
    dims = cfg["dims"]
    if args.stencil == 0 or args.rhs_tile <= 0 or args.traversal == 0:
        sys.exit("--pmc-probe needs an explicit --stencil, --rhs-tile and --traversal")
    lat = laph.Lattice(dims)
    lat.load_gauge(torch.from_numpy(ls.unit_gauge(dims)).cuda())
    lat.set_masses([cfg["masses"][0]], cfg["csw"])
    ms1, ms2 = lat.time_stages(args.prec, args.chunk, args.rhs_tile, 0, reps=3, stencil=args.stencil,
                               traversal=args.traversal)
    print("stage key %s sources %s: stage1 %.4f ms stage2 %.4f ms (3 timed launches each, after one warm "
          "launch)" % (stage_key(args, dims), stage_source_digest(), ms1, ms2), flush=True)
    x = torch.empty(2 ** 29, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print("copy: 3 x 2 GiB device-to-device", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="perambulator_32x32x32x64")
    ap.add_argument("--prec", default="f16n")
    ap.add_argument("--chunk", type=int, default=128)
    ap.add_argument("--rhs-tile", type=int, default=0, help="RHS per link load (0: autotuned)")
    ap.add_argument("--stencil", type=int, default=0, help="1 register RHS tiles, 2 LDS-staged links, 0 autotuned")
    ap.add_argument("--traversal", type=int, default=0, help="1 tiles of a site block together, 2 tile sweeps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--fp64-sample", type=int, default=4, help="RHS for the plain FP64 single-RHS comparison")
    ap.add_argument("--extra", action="store_true",
                    help="also measure the 16^3x32 single-RHS, 24^3x48 four-mass and gradient workloads")
    ap.add_argument("--laph-vectors", action="store_true",
                    help="only compute the LapH vectors of the 32^3x64 lattice (64 per timeslice) and print "
                         "their timing as one JSON line")
    ap.add_argument("--contractions", action="store_true",
                    help="only compute meson doublets and baryon triplets of 64 vectors on 32^3x64 for 4 "
                         "momenta and print their timing as one JSON line")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only launch the dominant stage (and a 2 GiB copy for the counter scale), for "
                         "rocprofv3 --pmc runs; needs --stencil, --rhs-tile and --traversal")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the perambulator path is measured on one MI355X "
              "(independent RHS batches would shard across GPUs with no collective)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2510_26313_amd as laph

    cfg = ls.CONFIGS[args.config]
    dims = cfg["dims"]
    if args.pmc_probe:
        pmc_probe(args, cfg, torch, laph)
        return
    if args.laph_vectors:
        print(json.dumps({"workload": "LapH vectors 32x32x32x64, 64 lowest eigenpairs of -Delta per timeslice, "
                                      "tol 1e-10", **laph_vectors_run(laph, torch)}), flush=True)
        return
    if args.contractions:
        print(json.dumps({"workload": "meson doublets and baryon triplets, 32x32x32x64, nev 64",
                          **contractions_run(laph, torch)}), flush=True)
        return
    nev = cfg["nev"]
    m0 = cfg["masses"][0]
    tol = 1e-10
    t_setup = time.perf_counter()
    U = ls.gauge_field(dims, cfg["seed_u"])
    V = ls.orthonormal_laph_vectors(dims, nev, cfg["seed_v"])
    lat = laph.Lattice(dims)
    lat.load_gauge(torch.from_numpy(U).cuda())
    lat.set_masses([m0], cfg["csw"])
    Vd = torch.from_numpy(V).cuda()
    v_src = np.ascontiguousarray(V[:, :1])
    del V
    if args.no_cpu_baseline:
        del U
    tuned = None
    if args.stencil == 0 or args.rhs_tile <= 0:
        # the library's autotuner picks the stencil form and RHS per link load for this batch
        tuned = lat.autotune(args.prec, args.chunk, 0)
        args.stencil, args.rhs_tile, args.traversal = tuned["stencil"], tuned["rhs_tile"], tuned["traversal"]
        # and the shape of the FP64 reliable-update stages (the solver reuses both choices)
        tuned["fp64_stages"] = lat.autotune("f64", args.chunk, 0)
    params = laph.default_params(inner_prec=args.prec, batched=1, chunk=args.chunk, rhs_tile=args.rhs_tile,
                                 stencil=args.stencil, traversal=args.traversal)
    setup_s = time.perf_counter() - t_setup
    t0s = cfg["t0s"]
    progress("setup done in %.1f s (autotuned: %s)" % (setup_s, tuned))

    for i in range(args.warmup):
        lat.perambulator_raw(Vd, t0s[i % len(t0s)], 0, tol, params)
        progress("warmup step %d done" % i)
    torch.cuda.synchronize()
    stats_all = []
    ms_solve = ms_proj = 0.0
    t_start = time.perf_counter()
    for i in range(args.steps):
        tau, st = lat.perambulator_raw(Vd, t0s[i % len(t0s)], 0, tol, params)
        tm = lat.timings()
        ms_solve += tm["solve_ms"]
        ms_proj += tm["project_ms"]
        stats_all += st
        progress("timed step %d done" % i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    n_rhs = args.steps * 4 * nev
    value = n_rhs / elapsed
    worst = max(s["true_res"] for s in stats_all)
    assert all(s["status"] == "converged" for s in stats_all) and worst <= tol, worst

    # the plain FP64 single-RHS solver on the same lattice, sources and tolerance (sampled RHS)
    fp64 = None
    if args.fp64_sample > 0:
        B = lat.make_sources(Vd[:, :1].contiguous(), t0s[0])[:args.fp64_sample].contiguous()
        p64 = laph.default_params(inner_prec="f64", batched=0, rhs_tile=1)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st64 = lat.solve_raw(B, 0, tol, p64)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        fp64 = {"rhs_per_s": round(args.fp64_sample / dt, 3), "sample_rhs": args.fp64_sample,
                "mean_iters": float(np.mean([s["iters"] for s in st64])),
                "max_true_res": max(s["true_res"] for s in st64),
                "speedup_of_batched_mixed": round(value / (args.fp64_sample / dt), 2)}
        del B

    progress("FP64 single-RHS comparison done")
    # projection: 8 flop per complex multiply-add, nev sinks x 4 spins x 3 colours x L^3 sites x T
    # timeslices per RHS
    proj_flops = 8.0 * nev * 4 * 3 * dims[0] * dims[1] * dims[2] * dims[3] * n_rhs
    # dominant kernels: the two fused stencil stages, timed with HIP events on the lattice stream
    ms1, ms2 = lat.time_stages(args.prec, args.chunk, args.rhs_tile, 0, reps=20, stencil=args.stencil,
                               traversal=args.traversal)
    vh = int(np.prod(dims)) // 2
    b1 = stage_bytes_per_site(args.prec, args.chunk, 1) * vh
    gbs1 = b1 / (ms1 * 1e-3) / 1e9
    fl1 = STAGE_FLOPS_PER_SITE_RHS * args.chunk * vh
    tfl1 = fl1 / (ms1 * 1e-3) / 1e12
    if tfl1 / ALU_PEAK_TFLOPS >= gbs1 / HBM_PEAK_GBS:
        roofline = {"bound": "alu", "achieved": round(tfl1, 3), "peak": round(ALU_PEAK_TFLOPS, 1),
                    "unit": "TFLOP/s", "frac": round(tfl1 / ALU_PEAK_TFLOPS, 4), "traffic": None}
    else:
        roofline = {"bound": "hbm", "achieved": round(gbs1, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs1 / HBM_PEAK_GBS, 4), "traffic": None}
    tb = stored_traffic(stage_key(args, dims))
    roofline["traffic"] = tb
    # the chip's FP32 vector figure counts packed FP32 FMAs, which this build does not emit
    roofline["peak_fp32_packed"] = 157.3
    roofline["frac_of_packed_peak"] = round(tfl1 / 157.3, 4)
    roofline.update({"kernel": "%s (stage 1: A_oo^-1 H_oe, %s, %d RHS per link load, %d RHS)"
                               % ("stage_lds_kernel" if args.stencil == 2 else "stage_kernel", args.prec,
                                  args.rhs_tile, args.chunk),
                     "ms_per_launch": round(ms1, 4), "algorithmic_bytes": b1, "hbm_gbs": round(gbs1, 1),
                     "hbm_frac": round(gbs1 / HBM_PEAK_GBS, 4), "tflops": round(tfl1, 3),
                     "stage2_ms_per_launch": round(ms2, 4)})

    # a plain device-to-device copy of 2 GiB: the HBM rate a streaming kernel reaches here
    xa = torch.empty(2 ** 29, dtype=torch.float32, device="cuda").fill_(1.0)
    xb = torch.empty_like(xa)
    xb.copy_(xa)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        xb.copy_(xa)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * xa.numel() * 4 * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del xa, xb
    # the stencil at small batches: HBM-bound at one RHS, at the FP32 ridge by eight
    # (algorithmic bytes and flops / time; register tiles up to 4 RHS, LDS links at 8)
    dslash = {"copy_gbs": round(copy_gbs, 1)}
    for prec, nrhs, st, tile in (("f32", 1, 1, 1), ("f16n", 1, 1, 1), ("f16n", 2, 1, 2), ("f16n", 4, 1, 4),
                                 ("f32", 8, 2, 8), ("f16n", 8, 2, 8)):
        m1, _ = lat.time_stages(prec, nrhs, tile, 0, reps=10, stencil=st, traversal=1)
        gb = stage_bytes_per_site(prec, nrhs, 1) * vh / (m1 * 1e-3) / 1e9
        tf = STAGE_FLOPS_PER_SITE_RHS * nrhs * vh / (m1 * 1e-3) / 1e12
        dslash["%s_nrhs%d" % (prec, nrhs)] = {"ms": round(m1, 4), "gbs": round(gb, 1),
                                              "hbm_frac": round(gb / HBM_PEAK_GBS, 4),
                                              "of_copy": round(gb / copy_gbs, 4), "tflops": round(tf, 2),
                                              "alu_frac": round(tf / ALU_PEAK_TFLOPS, 4)}

    out = {
        "metric": "perambulator RHS solved/s at rel. residual 1e-10; Dslash HBM GB/s vs peak",
        "value": round(value, 3), "unit": "RHS/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f16n/f32 inner, f64 outer", "data": "synthetic",
        "config": {"workload": "LapH perambulators %s, nev=%d, 4 source times x %d spin-diluted RHS, "
                               "m0=%g, c_sw=%g, batched BiCGStab chunks of %d, tol 1e-10, projection on "
                               "all %d sinks" % ("x".join(map(str, dims)), nev, 4 * nev, m0, cfg["csw"],
                                                  args.chunk, dims[3]),
                   "lattice": "x".join(map(str, dims)), "nev": nev, "rhs_per_step": 4 * nev,
                   "inner_prec": args.prec, "chunk": args.chunk, "rhs_tile": args.rhs_tile,
                   "stencil": "lds_links" if args.stencil == 2 else "register_tiles",
                   "traversal": "tile_sweeps" if args.traversal == 2 else "site_block_tiles"},
        "roofline": roofline,
        "detail": {"solve_ms": round(ms_solve, 1), "project_ms": round(ms_proj, 1),
                   "projection_tflops": round(proj_flops / (ms_proj * 1e-3) / 1e12, 2),
                   "projection_fp64_mfma_frac": round(proj_flops / (ms_proj * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS, 4),
                   "max_true_res": worst, "mean_iters": float(np.mean([s["iters"] for s in stats_all])),
                   "mean_updates": float(np.mean([s["updates"] for s in stats_all])),
                   "setup_s": round(setup_s, 1), "fp64_single_rhs": fp64, "autotuned": tuned,
                   "stage1_small_batches": dslash},
    }
    if args.extra:
        del tau, lat, Vd
        torch.cuda.empty_cache()
        out["detail"]["extra"] = extra_suite(laph, torch)
    if not args.no_cpu_baseline:
        progress("GPU measurements done; timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(cfg, dims, U, v_src, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
