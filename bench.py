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
# 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz
ALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
# flops per output site and RHS of a fused stage, the standard counts: the Wilson
# hop 1320 (per direction: spin projection 12, two SU(3) x colour-vector products
# 132, reconstruction and accumulation 24; the first accumulation is a copy) and
# two Hermitian 6x6 clover blocks 504
STAGE_FLOPS_PER_SITE_RHS = 1320 + 504


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


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, dims, U, V, t0):
    """The FP64 oracle timed on the host: one complete perambulator column of the
    headline workload -- the solve of one spin-diluted LapH source (k = 0, alpha = 0
    at source time t0) by the oracle's full-lattice BiCGStab to a relative residual
    of 1e-10, and its projection onto the LapH vectors of every sink timeslice --
    as RHS/s.  The clover term is built before the clock starts (the GPU's timed
    region also starts with it built)."""
    from oracle import dirac, laph as olaph, solvers
    m0, csw = cfg["masses"][0], cfg["csw"]
    D = dirac.WilsonClover(U, m0, csw)
    b = olaph.laph_sources(V[:, :1], t0)[:1]
    D.apply(b)   # first touch of the clover term
    t = time.perf_counter()
    x, info = solvers.bicgstab(D.apply, b, tol=1e-10)
    X4 = np.zeros((4,) + x.shape[1:], dtype=np.complex128)
    X4[0] = x[0]
    olaph.project(V, X4, 1)
    dt = time.perf_counter() - t
    cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    return {"value": 1.0 / dt, "unit": "RHS/s", "cores": cores, "kind": "oracle",
            "sample": "one complete perambulator column on %s: the FP64 oracle's full-lattice BiCGStab of the "
                      "LapH source k=0, alpha=0 at t0=%d to 1e-10 (%d iterations, %d restart(s), true residual "
                      "%.2e) and its projection on all %d sinks, %.1f s; OpenMP threads of the oracle's hop: %d"
                      % ("x".join(map(str, dims)), t0, int(info["iters"][0]), int(info["restarts"][0]),
                         float(info["true_res"][0]), dims[3], dt, cores),
            "seconds": round(dt, 2), "cpu_model": cpu_model(), "cpu_count": os.cpu_count()}


# The stencil sources whose counters a stored traffic figure describes.
STAGE_SOURCES = ["dslash_kernels.h", "dslash_lds.h", "laph_internal.h", "dslash_f16.hip", "dslash_f32.hip",
                 "dslash_f64.hip", "dslash.hip"]
PROFILES = os.path.join(ROOT, "profiles")


def stage_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in STAGE_SOURCES:
        with open(os.path.join(ROOT, "paper_2510_26313_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(key):
    """HBM bytes per launch of a stage shape from the committed counter summaries
    (lines ``traffic: key=... sources=... bytes_per_launch=...`` in profiles/*.md), or
    None when there is none for this shape or the stencil sources changed since the
    counters were taken."""
    digest = stage_source_digest()
    try:
        names = sorted(os.listdir(PROFILES))
    except OSError:
        return None
    for name in names:
        if not name.endswith(".md"):
            continue
        with open(os.path.join(PROFILES, name)) as fh:
            for ln in fh.read().splitlines():
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


def mg_run(laph, torch, masses, n_rhs=16, block=(4, 4, 4, 4), nvec=12, skip_mg=False, tol=1e-10):
    """The two-level multigrid against the batched FP16N BiCGStab on the 32^3 x 64 lattice:
    n_rhs spin-diluted LapH sources at t0 = 0 solved to 1e-10 at each mass of `masses`
    (the headline mass and lighter ones, where the plain solver needs many more
    iterations); times, iterations and RHS/s of both, and the multigrid setup time."""
    cfg = ls.CONFIGS["perambulator_32x32x32x64"]
    dims = cfg["dims"]
    lat = laph.Lattice(dims)
    lat.load_gauge(torch.from_numpy(ls.gauge_field(dims, cfg["seed_u"])).cuda())
    Vd = torch.from_numpy(ls.orthonormal_laph_vectors(dims, cfg["nev"], cfg["seed_v"])).cuda()
    B = lat.make_sources(Vd[:, :n_rhs // 4].contiguous(), 0)
    del Vd
    out = {"lattice": "x".join(map(str, dims)), "rhs": n_rhs, "block": list(block), "nvec": nvec}
    for m0 in masses:
        lat.set_masses([m0], cfg["csw"])
        tuned = lat.autotune("f16n", n_rhs, 0)
        lat.autotune("f64", n_rhs, 0)
        p = laph.default_params(inner_prec="f16n", stencil=tuned["stencil"], rhs_tile=tuned["rhs_tile"],
                                traversal=tuned["traversal"])
        (X, st), dt = _timed(torch, lambda: lat.solve_raw(B, 0, tol, p, raise_on_noconv=False))
        del X
        res = {"plain_f16n": _solve_summary(st, n_rhs, dt)}
        res["plain_f16n"]["converged"] = all(s["status"] == "converged" for s in st)
        res["plain_f16n"]["seconds"] = round(dt, 3)
        progress("m0 %g: plain batched solver %.2f s, %.1f iterations" % (m0, dt, res["plain_f16n"]["mean_iters"]))
        if not skip_mg:
            V0 = torch.from_numpy(ls.random_spinor((nvec,) + ls.spinor_shape(dims), 7300)).cuda()
            _, ts = _timed(torch, lambda: lat.mg_setup(V0, block, null_passes=4, null_tol=1e-2))
            del V0
            lat.mg_solve(B[:1].contiguous(), tol)   # warm
            (X, st), dt = _timed(torch, lambda: lat.mg_solve(B, tol, allow_noconv=True))
            del X
            res["multigrid"] = _solve_summary(st, n_rhs, dt)
            res["multigrid"]["converged"] = all(s["status"] == "converged" for s in st)
            res["multigrid"].update({"seconds": round(dt, 3), "setup_seconds": round(ts, 3),
                                     "fp64_residual_recomputations": float(np.mean([s["updates"] for s in st]))})
            res["multigrid_over_plain"] = round(res["plain_f16n"]["seconds"] / dt, 3)
            progress("m0 %g: multigrid %.2f s (setup %.2f s), %.1f iterations" % (m0, dt, ts,
                                                                                 res["multigrid"]["mean_iters"]))
        out["m0=%g" % m0] = res
        lat.release_scratch()
        torch.cuda.empty_cache()
    return out


# Stage shapes whose counters the probe collects: the bench's dominant shape (128 RHS,
# LDS links x16, tile sweeps) and the bandwidth-bound small batches, each in its fastest
# measured form (2 RHS: register tiles of 1; 4 RHS: LDS links x4, 22 % faster than register
# tiles of 4; 8 RHS: LDS links x8).
PROBE_SHAPES = [("f16n", 128, 2, 16, 2), ("f32", 1, 1, 1, 1), ("f16n", 1, 1, 1, 1), ("f16n", 2, 1, 1, 1),
                ("f16n", 4, 2, 4, 1), ("f32", 8, 2, 8, 1), ("f16n", 8, 2, 8, 1)]


def stage_key(dims, prec, nrhs, stencil, tile, traversal, stage):
    return "%s/%s/n%d/s%d/t%d/v%d/stage%d" % ("x".join(map(str, dims)), prec, nrhs, stencil, tile, traversal, stage)


def pmc_probe(args, cfg, torch, laph):
    """Launch the stage shapes of PROBE_SHAPES (unit gauge: the traffic does not depend
    on the values), each stage 1 and stage 2 once to warm and three times timed, then
    three streaming copies of 2 GiB with the library's copy kernel that calibrate the
    byte counters, for hardware-counter runs."""
    dims = cfg["dims"]
    lat = laph.Lattice(dims)
    lat.load_gauge(torch.from_numpy(ls.unit_gauge(dims)).cuda())
    lat.set_masses([cfg["masses"][0]], cfg["csw"])
    for prec, n, st, tile, trav in PROBE_SHAPES:
        ms1, ms2 = lat.time_stages(prec, n, tile, 0, reps=3, stencil=st, traversal=trav)
        print("probe %s %s sources %s: stage1 %.4f ms stage2 %.4f ms (3 timed launches each after one warm "
              "launch)" % (stage_key(dims, prec, n, st, tile, trav, 1), stage_key(dims, prec, n, st, tile, trav, 2),
                           stage_source_digest(), ms1, ms2), flush=True)
        lat.release_scratch()
    x = torch.empty(2 ** 29, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    ms = lat.stream_copy(y, x, reps=2)
    print("copy: stream_copy_kernel, 1 warm + 2 timed copies of 2 GiB, %.4f ms each" % ms, flush=True)


def copy_peak(lat, torch, gib=4):
    """Read + write GB/s of the library's streaming copy of a gib GiB buffer."""
    n = (gib << 30) // 4
    xa = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
    xb = torch.empty_like(xa)
    ms = lat.stream_copy(xb, xa, reps=5)
    del xa, xb
    torch.cuda.empty_cache()
    return 2.0 * (gib << 30) / (ms * 1e-3) / 1e9, ms


def copy_same_bytes_ms(lat, torch, nbytes, reps=10):
    """ms of the library's streaming copy that reads and writes nbytes in all (nbytes / 2
    each way): the ceiling for a bandwidth-bound launch moving the same bytes, launch and
    ramp included."""
    n = max(16, (int(nbytes) // 2) // 16 * 16) // 4
    xa = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
    xb = torch.empty_like(xa)
    ms = lat.stream_copy(xb, xa, reps=reps)
    del xa, xb
    return ms


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
    ap.add_argument("--fp64-sample", type=int, default=4, help="RHS for the plain FP64 single-RHS comparison")
    ap.add_argument("--extra", action="store_true",
                    help="also measure the 16^3x32 single-RHS, 24^3x48 four-mass and gradient workloads")
    ap.add_argument("--laph-vectors", action="store_true",
                    help="only compute the LapH vectors of the 32^3x64 lattice (64 per timeslice) and print "
                         "their timing as one JSON line")
    ap.add_argument("--contractions", action="store_true",
                    help="only compute meson doublets and baryon triplets of 64 vectors on 32^3x64 for 4 "
                         "momenta and print their timing as one JSON line")
    ap.add_argument("--mg", action="store_true",
                    help="only compare the two-level multigrid with the batched FP16N solver on 32x32x32x64 "
                         "(16 LapH sources, 1e-10) at the masses of --mg-masses; one JSON line")
    ap.add_argument("--mg-masses", default="0.02,-0.4", help="comma-separated bare masses for --mg")
    ap.add_argument("--mg-rhs", type=int, default=16, help="RHS for --mg (a multiple of 4)")
    ap.add_argument("--mg-skip", action="store_true", help="--mg: time the plain solver only")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only launch the stage shapes whose counters are kept (and a 2 GiB copy for the "
                         "counter scale), for rocprofv3 --pmc runs")
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
    if args.mg:
        masses = [float(m) for m in args.mg_masses.split(",")]
        print(json.dumps({"workload": "multigrid vs batched FP16N BiCGStab, 32x32x32x64, %d LapH sources, tol 1e-10"
                                      % args.mg_rhs, **mg_run(laph, torch, masses, args.mg_rhs, skip_mg=args.mg_skip)}),
              flush=True)
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
    if args.no_cpu_baseline:
        del U, V
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
    shape = (args.prec, args.chunk, args.stencil, args.rhs_tile, args.traversal)
    copy_gbs, copy_ms = copy_peak(lat, torch)

    def stage_figures(ms, stage, sh):
        prec, n = sh[0], sh[1]
        b = stage_bytes_per_site(prec, n, stage) * vh
        fl = STAGE_FLOPS_PER_SITE_RHS * n * vh
        gbs, tfl = b / (ms * 1e-3) / 1e9, fl / (ms * 1e-3) / 1e12
        tb = stored_traffic(stage_key(dims, *sh, stage))
        f = {"ms_per_launch": round(ms, 4), "algorithmic_bytes": b, "hbm_gbs": round(gbs, 1),
             "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "of_copy": round(gbs / copy_gbs, 4), "tflops": round(tfl, 3),
             "alu_frac": round(tfl / ALU_PEAK_TFLOPS, 4), "counter_bytes": tb,
             "counter_gbs": round(tb / (ms * 1e-3) / 1e9, 1) if tb else None}
        return f, gbs, tfl, tb

    f1, gbs1, tfl1, tb1 = stage_figures(ms1, 1, shape)
    f2, _, _, _ = stage_figures(ms2, 2, shape)
    if tfl1 / ALU_PEAK_TFLOPS >= gbs1 / HBM_PEAK_GBS:
        roofline = {"bound": "alu", "achieved": round(tfl1, 3), "peak": round(ALU_PEAK_TFLOPS, 1),
                    "unit": "TFLOP/s", "frac": round(tfl1 / ALU_PEAK_TFLOPS, 4), "traffic": tb1}
    else:
        roofline = {"bound": "hbm", "achieved": round(gbs1, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs1 / HBM_PEAK_GBS, 4), "traffic": tb1}
    # the chip's FP32 vector figure counts packed FP32 FMAs, which this build does not emit
    roofline["peak_fp32_packed"] = 157.3
    roofline["frac_of_packed_peak"] = round(tfl1 / 157.3, 4)
    roofline.update({"kernel": "%s (stage 1: A_oo^-1 H_oe, %s, %d RHS per link load, %d RHS)"
                               % ("stage_lds_kernel" if args.stencil == 2 else "stage_kernel", args.prec,
                                  args.rhs_tile, args.chunk),
                     "flops_per_site_rhs": STAGE_FLOPS_PER_SITE_RHS, "stage1": f1, "stage2": f2,
                     "stage2_alu_frac": f2["alu_frac"],
                     "copy_kernel_gbs": round(copy_gbs, 1), "copy_kernel_ms_4gib": round(copy_ms, 3)})

    # the stencil at small batches: HBM-bound at one RHS, near the FP32 ridge by eight
    # (algorithmic bytes and flops / time; counter bytes where committed for this build)
    # of_copy_same_bytes: against a copy of the same algorithmic bytes (a 0.1-1 ms launch
    # does not reach the 4 GiB copy's rate: launch and ramp are a larger share)
    dslash = {"copy_kernel_gbs": round(copy_gbs, 1)}
    for sh in PROBE_SHAPES[1:]:
        m1, m2 = lat.time_stages(sh[0], sh[1], sh[3], 0, reps=10, stencil=sh[2], traversal=sh[4])
        lat.release_scratch()
        entry = {}
        for st, ms in ((1, m1), (2, m2)):
            f = stage_figures(ms, st, sh)[0]
            cms = copy_same_bytes_ms(lat, torch, f["algorithmic_bytes"])
            f["copy_same_bytes_ms"] = round(cms, 4)
            f["of_copy_same_bytes"] = round(cms / ms, 4)
            entry["stage%d" % st] = f
        dslash["%s_nrhs%d" % (sh[0], sh[1])] = entry
    torch.cuda.empty_cache()

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
        lat.release_scratch()
        torch.cuda.empty_cache()
        out["detail"]["extra"] = extra_suite(laph, torch)
    if not args.no_cpu_baseline:
        progress("GPU measurements done; timing the CPU oracle")
        del tau, Vd
        lat.release_scratch()
        out["cpu_baseline"] = cpu_baseline(cfg, dims, U, V, t0s[0])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
