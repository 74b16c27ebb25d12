"""Parity at the benchmark sizes, in the configuration bench.py times.

The oracle cannot solve 32^3 x 64 (or 24^3 x 48) in test time, so these checks
use outputs it computes one by one and properties that hold at any size:

* the perambulator workload (32^3 x 64, nev 64, m0 0.02): the fused perambulator for t0 = 0 and t0 = 1
  (FP16N inner, LDS stencil, chunks of 128 -- the bench configuration) obeys
  gamma5 reciprocity between the two source times; a perambulator over 8 LapH
  vectors and a solve of the same sources made with the same parameters give
  solutions that pass the oracle's D at sampled sites (pointwise residual) and
  whose oracle projection reproduces the sampled tau entries;
* the multi-mass workload (24^3 x 48, four masses split 40/72/64/80 in one batched solve): per-RHS
  FP64 residual reported by the library and the oracle's D at sampled sites;
* the single-RHS workload (16^3 x 32, single-RHS solver, FP32 and FP16N inner): sampled RHS against
  full oracle solves (1e-8).
"""
import numpy as np
import pytest
import torch

import laph_synth as ls
from gpu_common import dev, host, log_case, make_lattice, per_rhs_rel, require_gpu
from oracle import dirac, laph, solvers

pytestmark = pytest.mark.gpu


def _sample_sites(dims, n, seed, t_fixed=None):
    lx, ly, lz, lt = dims
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        t = int(rng.integers(0, lt)) if t_fixed is None else t_fixed
        out.append((t, int(rng.integers(0, lz)), int(rng.integers(0, ly)), int(rng.integers(0, lx))))
    return out


def _pointwise_residual(U, X, B, sites, m0, csw):
    DX = dirac.apply_at_sites(U, X, sites, m0, csw)
    b = np.stack([B[:, t, z, y, x] for (t, z, y, x) in sites], axis=1)
    return np.abs(b - DX).max(axis=(1, 2, 3)), np.linalg.norm(B.reshape(B.shape[0], -1), axis=1)


@pytest.fixture()
def peramb_case():
    require_gpu()
    cfg = ls.CONFIGS["perambulator_32x32x32x64"]
    dims = cfg["dims"]
    log_case("32^3x64 inputs", dims=dims)
    U = ls.gauge_field(dims, cfg["seed_u"])
    V = ls.orthonormal_laph_vectors(dims, cfg["nev"], cfg["seed_v"])
    lat = make_lattice(dims, U, masses=cfg["masses"], csw=cfg["csw"])
    return dict(cfg=cfg, U=U, V=V, lat=lat, Vd=dev(V))


def test_perambulator_32x32x32x64_sampled_and_reciprocal(peramb_case):
    import paper_2510_26313_amd as pl
    cfg, U, V, lat, Vd = peramb_case["cfg"], peramb_case["U"], peramb_case["V"], peramb_case["lat"], peramb_case["Vd"]
    m0, csw = cfg["masses"][0], cfg["csw"]
    p = pl.default_params(inner_prec="f16n", chunk=128, rhs_tile=16, stencil=2)
    log_case("32^3x64 perambulator", t0=0)
    tauA, stA = lat.perambulator_raw(Vd, 0, 0, 1e-10, p)
    log_case("32^3x64 perambulator", t0=1)
    tauB, stB = lat.perambulator_raw(Vd, 1, 0, 1e-10, p)
    assert all(s["status"] == "converged" and s["true_res"] <= 1e-10 for s in stA + stB)
    tauA, tauB = host(tauA), host(tauB)
    # gamma5 reciprocity between source times 0 and 1.  Each side comes from its
    # own solves, good to about cond(D) * 1e-10 in absolute terms, so the check
    # uses neighbouring source times, where these entries are large (at a time
    # separation of 16 they are ~1e-6 of the source-slice entries and the
    # relative agreement of two independent 1e-10 solves drops to ~1e-6).
    g5 = np.array([1, 1, -1, -1])
    exp = np.einsum("b,a,klab->lkba", g5, g5, np.conj(tauB[0]))
    assert np.linalg.norm(tauA[1] - exp) <= 1e-8 * np.linalg.norm(exp)
    # sampled solutions.  Two independent solves to a relative residual of 1e-10
    # agree only to about cond(D) * 1e-10, so the oracle's projection is checked
    # on the very solves the perambulator made: a perambulator over the first 8
    # LapH vectors (32 RHS = one chunk of 32) and a solve of the same 32 sources
    # with the same parameters run the same per-RHS arithmetic.
    nev8 = 8
    V8 = np.ascontiguousarray(V[:, :nev8])
    p32 = pl.default_params(inner_prec="f16n", chunk=32, rhs_tile=16, stencil=2)
    log_case("32^3x64 perambulator", t0=0, nev=nev8, chunk=32)
    tauC, stC = lat.perambulator_raw(dev(V8), 0, 0, 1e-10, p32)
    tauC = host(tauC)
    rhs = [5, 18, 31]
    B = laph.laph_sources(V8, 0)
    log_case("32^3x64 sampled solves", nrhs=B.shape[0])
    Xd, st = lat.solve_raw(dev(B), 0, 1e-10, p32)
    X = host(Xd[rhs])
    del Xd
    assert [s["iters"] for s in st] == [s["iters"] for s in stC]
    sites = _sample_sites(cfg["dims"], 24, 7) + _sample_sites(cfg["dims"], 8, 8, t_fixed=0)
    res, bn = _pointwise_residual(U, X, B[rhs], sites, m0, csw)
    assert np.all(res <= 1e-10 * bn)
    for i, r in enumerate(rhs):
        k, al = divmod(r, 4)
        for t in (0, 1, 33, 63):
            # tau[t][l][k][beta][alpha] for this RHS from the oracle's projection of X;
            # |V_t^dagger X_t| <= |X_t| bounds the rounding of either sum
            exp_t = np.einsum("lzyxa,zyxba->lb", np.conj(V8[t]), X[i, t])
            got = tauC[t, :, k, :, al]
            assert np.linalg.norm(got - exp_t) <= 1e-12 * np.linalg.norm(X[i, t])
        # the first 8 sinks of the bench-shaped perambulator agree to the solve accuracy
        assert np.linalg.norm(tauA[0, :nev8, k, :, al] - tauC[0, :, k, :, al]) <= 1e-6 * np.linalg.norm(tauC[0, :, k, :, al])


def test_multimass_24x24x24x48_batched_sampled():
    import gc
    import paper_2510_26313_amd as pl
    require_gpu()
    gc.collect()
    torch.cuda.empty_cache()
    cfg = ls.CONFIGS["multimass_24x24x24x48"]
    dims = cfg["dims"]
    log_case("24^3x48 inputs", dims=dims)
    U = ls.gauge_field(dims, cfg["seed_u"])
    V = ls.orthonormal_laph_vectors(dims, cfg["nev"], cfg["seed_v"])
    lat = make_lattice(dims, U, masses=cfg["masses"], csw=cfg["csw"])
    mi = ls.rhs_masses(cfg)
    Vd = dev(V)
    B = lat.make_sources(Vd, 0)
    log_case("24^3x48 batched solve", nrhs=len(mi))
    X, st = lat.solve_raw(B, mi, 1e-10, pl.default_params(inner_prec="f16n", rhs_tile=16, stencil=2))
    assert all(s["status"] == "converged" and s["true_res"] <= 1e-10 for s in st)
    iters = {m: [s["iters"] for s, mm in zip(st, mi) if mm == m] for m in range(4)}
    print("24^3x48 iterations per mass", {cfg["masses"][m]: (min(v), max(v)) for m, v in iters.items()}, flush=True)
    pick = [0, 39, 40, 111, 112, 175, 176, 255]   # two per mass, at the range edges
    Xs, Bs = host(X[pick]), host(B[pick])
    del X
    sites = _sample_sites(dims, 16, 11) + _sample_sites(dims, 8, 12, t_fixed=0)
    for j, r in enumerate(pick):
        res, bn = _pointwise_residual(U, Xs[j:j + 1], Bs[j:j + 1], sites, cfg["masses"][mi[r]], cfg["csw"])
        assert res[0] <= 1e-10 * bn[0]


@pytest.fixture(scope="module")
def single_case():
    require_gpu()
    cfg = ls.CONFIGS["single_rhs_16x16x16x32"]
    dims = cfg["dims"]
    U = ls.gauge_field(dims, cfg["seed_u"])
    V = ls.orthonormal_laph_vectors(dims, cfg["nev"], cfg["seed_v"])
    B = laph.laph_sources(V, 0)[[0, 77]]
    log_case("16^3x32 oracle solves", nrhs=2)
    D = dirac.WilsonClover(U, cfg["masses"][0], cfg["csw"])
    x_ref, _ = solvers.bicgstab(D.apply, B, tol=1e-13)
    lat = make_lattice(dims, U, masses=cfg["masses"], csw=cfg["csw"])
    return dict(B=B, x_ref=x_ref, lat=lat)


@pytest.mark.parametrize("prec", ["f32", "f16n"])
def test_single_rhs_16x16x16x32_vs_oracle(single_case, prec):
    import paper_2510_26313_amd as pl
    log_case("16^3x32 single-rhs", prec=prec)
    X, st = single_case["lat"].solve_raw(dev(single_case["B"]), 0, 1e-10, pl.default_params(inner_prec=prec, batched=0))
    assert per_rhs_rel(host(X), single_case["x_ref"]).max() < 1e-8
    assert all(s["status"] == "converged" and s["true_res"] <= 1e-10 for s in st)


def _odd_even_sites(dims, n, seed, parity):
    lx, ly, lz, lt = dims
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        t, z, y = int(rng.integers(0, lt)), int(rng.integers(0, lz)), int(rng.integers(0, ly))
        x = int(rng.integers(0, lx // 2)) * 2
        x += (parity + t + z + y + x) % 2
        out.append((t, z, y, x))
    return out


@pytest.mark.parametrize("prec,tol", [("f32", 1e-6), ("f16n", 3e-3)])
def test_stages_32x32x32x64_128rhs_sampled(prec, tol):
    """The bench's dominant launches at full size: 128 RHS of one mass, links staged in
    LDS with 16 RHS per link load, each tile sweeping the lattice.  Inputs are seeded
    combinations of four random base fields (RHS r: sum_k c_rk B_k), so the oracle's
    one-site hop and clover inverse give the expected output of any sampled (RHS, site);
    stage 2's fused <y, out> of sampled RHS is checked against an FP64 dot of the
    kernel's own stored output."""
    import gc
    import torch
    require_gpu()
    gc.collect()
    torch.cuda.empty_cache()
    cfg = ls.CONFIGS["perambulator_32x32x32x64"]
    dims, m0, csw, n = cfg["dims"], cfg["masses"][0], cfg["csw"], 128
    U = ls.gauge_field(dims, cfg["seed_u"])
    lat = make_lattice(dims, U, masses=cfg["masses"], csw=csw)
    base = ls.random_spinor(ls.spinor_shape(dims, 4), 7200)
    rng = np.random.default_rng(7201)
    c_in = rng.standard_normal((n, 4)) + 1j * rng.standard_normal((n, 4))
    c_y = 0.3 * (rng.standard_normal((n, 4)) + 1j * rng.standard_normal((n, 4)))
    base_d = dev(base).reshape(4, -1)
    per = lat.field_bytes(prec, 1)
    bufs = {}
    for name, coef, parity in (("e_in", c_in, 0), ("o_in", c_in, 1), ("y", c_y, 0)):
        buf = torch.empty(per * n, dtype=torch.uint8, device="cuda")
        for r0 in range(0, n, 8):
            chunk = torch.matmul(dev(coef[r0:r0 + 8]), base_d).reshape(lat.spinor_shape(8))
            lat.pack(chunk, prec, parity=parity, out=buf, rhs_offset=r0)
            del chunk
        bufs[name] = buf
    del base_d
    kw = dict(prec=prec, stencil=2, rhs_tile=16, traversal=2)
    log_case("32^3x64 stage 1, 128 RHS", prec=prec)
    o1, _ = lat.apply_stage(1, bufs["e_in"], n, **kw)
    log_case("32^3x64 stage 2, 128 RHS", prec=prec)
    o2, d2 = lat.apply_stage(2, bufs["o_in"], n, y=bufs["y"], w=bufs["y"], **kw)
    assert np.all(np.isfinite(d2)) and np.all(np.abs(d2[:, 0]) > 0)
    sites1 = _odd_even_sites(dims, 12, 7202, 1)
    sites2 = _odd_even_sites(dims, 12, 7203, 0)
    h1 = dirac.hop_at_sites(U, base, sites1)      # [k][site][4][3]; odd sites read even neighbours only
    h2 = dirac.hop_at_sites(U, base, sites2)
    ai1 = [dirac.clover_inverse_at(U, s, m0, csw) for s in sites1]
    ai2 = [dirac.clover_inverse_at(U, s, m0, csw) for s in sites2]
    for r in (0, 15, 16, 77, 127):
        g1 = host(lat.unpack(lat.field_slice(o1, prec, r), 1, prec, parity=1))[0]
        g2 = host(lat.unpack(lat.field_slice(o2, prec, r), 1, prec, parity=0))[0]
        yr = host(lat.unpack(lat.field_slice(bufs["y"], prec, r), 1, prec, parity=0))[0]
        got1 = np.stack([g1[s] for s in sites1])
        got2 = np.stack([g2[s] for s in sites2])
        exp1 = np.stack([(ai1[i] @ np.tensordot(c_in[r], h1[:, i], 1).reshape(12)).reshape(4, 3)
                         for i in range(len(sites1))])
        ysite = np.stack([np.tensordot(c_y[r], base[:, t, z, y, x], 1) for (t, z, y, x) in sites2])
        exp2 = np.stack([ysite[i] - 0.25 * (ai2[i] @ np.tensordot(c_in[r], h2[:, i], 1).reshape(12)).reshape(4, 3)
                         for i in range(len(sites2))])
        assert np.linalg.norm(got1 - exp1) < tol * np.linalg.norm(exp1), r
        assert np.linalg.norm(got2 - exp2) < tol * np.linalg.norm(exp2), r
        own = np.vdot(yr, g2)
        bound = (tol if prec == "f32" else 3e-3) * np.linalg.norm(yr) * np.linalg.norm(g2)
        assert abs(d2[r, 0] + 1j * d2[r, 1] - own) <= bound, r
    del bufs, o1, o2
    torch.cuda.empty_cache()
