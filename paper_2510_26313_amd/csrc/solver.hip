// Host orchestration of the even-odd mixed-precision (batched) BiCGStab.
//
// Per batch of right-hand sides ("slots"):
//   1. sources -> FP64 even/odd halves, |B|^2, even-odd prepared source b_hat
//   2. r64 = b_hat - M_hat x64 (FP64), r = lower(r64), r^ = r
//   3. iterations in the inner precision; every kernel reads its scalars from
//      device memory and the finalize kernels compute alpha, omega, rho, beta
//      and the reliable-update decision on the device; updates (x64 += x_lo,
//      FP64 true residual, r = lower(r64)) are masked per slot inside the same
//      launch sequence, so one captured HIP graph of K iterations serves every
//      replay; the host only polls the per-slot status every K iterations and
//      compacts the tile table when slots have finished
//   4. odd reconstruction, FP64 full-lattice residual |B - D X| per slot
// The paper batches solves so that the stencil coefficients are reused across
// the batch (Sec. "Batched Linear Solves") and runs its sparse work in mixed
// precision (Sec. "QUDA").
#include <algorithm>
#include <cmath>
#include <cstring>

#include "laph_solver.h"

namespace laph {

// RHS per register tile: 4, 2 or 1
static int reg_tile(int ns) { return ns >= 4 ? 4 : (ns >= 2 ? 2 : 1); }

// Stencil form and tile size of the inner iterations when the caller fixes them
// or no tuned choice exists: FP64 keeps the register tiles (its LDS link stage
// would need twice the LDS); FP32 / FP16N use the LDS-staged links with up to
// 16 RHS sharing each link load.
void Solver::choose_shape(const laph_solve_params &p, int ns, int &form, int &nr, int &form64, int &nr64) {
    const int prec = p.inner_prec;
    form = prec == LAPH_F64 ? kFormRegister : kFormLds;
    if (p.stencil == 1) form = kFormRegister;
    if (p.stencil == 2) form = kFormLds;
    if (form == kFormLds)
        nr = p.rhs_tile > 0 ? p.rhs_tile : (ns >= 16 ? 16 : (ns >= 8 ? 8 : 4));
    else
        nr = p.rhs_tile > 0 ? p.rhs_tile : reg_tile(ns);
    if (prec == LAPH_F64) {
        form64 = form;
        nr64 = nr;
        return;
    }
    form64 = p.stencil64 == 2 ? kFormLds : kFormRegister;
    if (form64 == kFormLds)
        nr64 = p.rhs_tile64 > 0 ? p.rhs_tile64 : (ns >= 8 ? 8 : 4);
    else
        nr64 = p.rhs_tile64 > 0 ? p.rhs_tile64 : reg_tile(ns);
}

// The integer tables are sized for the largest tiles (16 RHS), so the workspace
// does not depend on the tuned shapes.
static size_t table_ints(int ns) { return 3 * (size_t)ns * 16 + 6 * (size_t)ns + 16; }

size_t Solver::layout(const Ctx &c, int ns, int prec, char *base, WS *ws) {
    const size_t h64 = c.hv(LAPH_F64), hlo = c.hv(prec), hx = c.hv(prec == LAPH_F64 ? LAPH_F64 : LAPH_F32);
    const int pstride = partial_stride(c);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += round256(bytes);
        return o;
    };
    auto op = [&](size_t o, size_t stride) {
        Operand r;
        r.base = base ? base + o : nullptr;
        r.stride = stride;
        return r;
    };
    WS w;
    w.E0 = op(take(ns * h64), h64);
    w.E1 = op(take(ns * h64), h64);
    w.E2 = op(take(ns * h64), h64);
    w.O0 = op(take(ns * h64), h64);
    w.O1 = op(take(ns * h64), h64);
    // r, rh, p, v are contiguous: the autotuner uses them as its 4 * ns fields
    w.r = op(take(ns * hlo), hlo);
    w.rh = op(take(ns * hlo), hlo);
    w.p = op(take(ns * hlo), hlo);
    w.v = op(take(ns * hlo), hlo);
    w.t = op(take(ns * hlo), hlo);
    w.tmp = op(take(ns * hlo), hlo);
    w.x = op(take(ns * hx), hx);
    size_t o_st = take(ns * sizeof(SlotState));
    size_t o_part = take((size_t)ns * 3 * pstride * sizeof(double));
    const size_t nints = std::max(table_ints(ns), tune_ints(ns));
    size_t o_ints = take(nints * sizeof(int));
    if (ws && base) {
        w.st = reinterpret_cast<SlotState *>(base + o_st);
        w.partials = reinterpret_cast<double *>(base + o_part);
        w.ints = reinterpret_cast<int *>(base + o_ints);
        w.nints = nints;
        *ws = w;
    }
    return off;
}

// carve the tile tables for the chosen tile sizes out of the integer region
void Solver::carve_tables() {
    int *ints = ws.ints;
    ws.tile_slots = ints;
    ws.tile_mass = ws.tile_slots + (size_t)ns * nr;
    ws.tile64_slots = ws.tile_mass + ns;
    ws.tile64_mass = ws.tile64_slots + (size_t)ns * nr64;
    ws.list = ws.tile64_mass + ns;
    ws.slot_mass = ws.list + ns;
    ws.ntiles = ws.slot_mass + ns;
    ws.nlist = ws.ntiles + 1;
    ws.ntiles64 = ws.ntiles + 2;
    // device-built tables (not uploaded): flagged FP64 tiles and slots
    ws.tile64f_slots = ws.ntiles + 4;
    ws.tile64f_mass = ws.tile64f_slots + (size_t)ns * nr64;
    ws.flist = ws.tile64f_mass + ns;
    ws.ntiles64f = ws.flist + ns;
    ws.nflist = ws.ntiles64f + 1;
    ws.nints_used = (size_t)(ws.ntiles + 3 - ints);
}

size_t solver_workspace_bytes(const Ctx &c, int nslots, const laph_solve_params &p) {
    return Solver::layout(c, nslots, p.inner_prec, nullptr, nullptr);
}

laph_status Solver::init(Ctx &ctx, int nslots, const laph_solve_params &params, char *work, size_t bytes,
                         int tune_mass) {
    c = &ctx;
    p = params;
    ns = nslots;
    prec = p.inner_prec;
    const size_t need = layout(ctx, ns, prec, nullptr, nullptr);
    if (!work || bytes < need)
        return set_error(LAPH_ERR_WORKSPACE, "solver workspace too small: %zu < %zu bytes", bytes, need);
    layout(ctx, ns, prec, work, &ws);
    choose_shape(p, ns, form, nr, form64, nr64);
    site_major = p.traversal == 2 ? 1 : 0;
    site_major64 = prec == LAPH_F64 ? site_major : 0;
    // autotuned shapes: reuse a choice for this (precision, batch) or measure one now,
    // for the inner iterations and for the FP64 stages of the reliable updates
    // (timed on the FP64 half-vectors E0..O0, not in use yet)
    // found: whether a choice exists (errors of the tuning runs are returned)
    auto shape_of = [&](int pr, char *fields, Ctx::Shape &out, bool &found) -> laph_status {
        auto it = ctx.tuned.find({pr, ns});
        if (it == ctx.tuned.end() && tune_mass >= 0) {
            Ctx::Shape sh{};
            LAPH_TRY(autotune_stencil(ctx, pr, ns, tune_mass, fields, ws.partials, ws.ints, &sh, nullptr));
            it = ctx.tuned.find({pr, ns});
        }
        found = it != ctx.tuned.end();
        if (found) out = it->second;
        return LAPH_OK;
    };
    Ctx::Shape sh{};
    bool found = false;
    if (p.stencil == 0 && p.rhs_tile <= 0) {
        LAPH_TRY(shape_of(prec, prec == LAPH_F64 ? ws.E0.base : ws.r.base, sh, found));
        if (found) {
            form = sh.form;
            nr = sh.tile;
            if (p.traversal == 0) site_major = sh.site_major;
            if (prec == LAPH_F64) {
                form64 = form;
                nr64 = nr;
                site_major64 = site_major;
            }
        }
    }
    if (prec != LAPH_F64 && p.stencil64 == 0 && p.rhs_tile64 <= 0) {
        LAPH_TRY(shape_of(LAPH_F64, ws.E0.base, sh, found));
        if (found) {
            form64 = sh.form;
            nr64 = sh.tile;
            site_major64 = sh.site_major;
        }
    }
    for (int k = 0; k < 2; ++k) {
        const int f = k ? form64 : form, t = k ? nr64 : nr;
        if (f == kFormRegister && t != 1 && t != 2 && t != 4)
            return set_error(LAPH_ERR_INVALID, "rhs_tile must be 1, 2 or 4 for register tiles");
        if (f == kFormLds && t != 4 && t != 8 && t != 16)
            return set_error(LAPH_ERR_INVALID, "rhs_tile must be 4, 8 or 16 for LDS-staged links");
    }
    carve_tables();
    // grouping by mass adds at most one partly filled tile per extra mass
    const int nm = std::max(1, ctx.n_mass);
    tiles_cap = std::min(ns, (ns + nr - 1) / nr + nm - 1);
    tiles64_cap = std::min(ns, (ns + nr64 - 1) / nr64 + nm - 1);
    nsb256 = stage_nsb(ctx, kFormRegister);
    nsb_inner = stage_nsb(ctx, form);
    nsb64 = stage_nsb(ctx, form64);
    pstride = partial_stride(ctx);
    host_ints.assign(ws.nints_used, 0);
    host_st.assign(ns, SlotState{});
    return LAPH_OK;
}

Solver::~Solver() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
}

BlasArgs Solver::blas(int list_max) const {
    BlasArgs a;
    a.vh = c->g.vh;
    a.nsb = nsb256;
    a.pstride = pstride;
    a.list = ws.list;
    a.nlist = ws.nlist;
    a.nlist_max = list_max;
    a.st = ws.st;
    a.partials = ws.partials;
    a.r = ws.r;
    a.rh = ws.rh;
    a.p = ws.p;
    a.v = ws.v;
    a.t = ws.t;
    a.x = ws.x;
    a.x64 = ws.E1;
    a.r64 = ws.E2;
    a.flist = ws.flist;
    a.nflist = ws.nflist;
    return a;
}

FinArgs Solver::fin(int list_max, int nsb) const {
    FinArgs f;
    f.list = ws.list;
    f.nlist = ws.nlist;
    f.nlist_max = list_max;
    f.nsb = nsb > 0 ? nsb : nsb256;
    f.pstride = pstride;
    f.st = ws.st;
    f.partials = ws.partials;
    return f;
}

Tiles Solver::tiles(bool f64, bool flagged) const {
    Tiles t;
    if (f64 && flagged) {
        t.slots = ws.tile64f_slots;
        t.mass = ws.tile64f_mass;
        t.ntiles = ws.ntiles64f;
    } else {
        t.slots = f64 ? ws.tile64_slots : ws.tile_slots;
        t.mass = f64 ? ws.tile64_mass : ws.tile_mass;
        t.ntiles = f64 ? ws.ntiles64 : ws.ntiles;
    }
    t.ntiles_max = f64 ? tiles64_cap : tiles_cap;
    t.nr = f64 ? nr64 : nr;
    return t;
}

// Upload the slot list and the tile tables (inner form and FP64) for the given slots,
// grouped by mass so that every tile shares one clover inverse.
laph_status Solver::upload_tables(const std::vector<int> &slots) {
    std::vector<int> sorted = slots;
    std::stable_sort(sorted.begin(), sorted.end(), [&](int a, int b) { return mass[a] < mass[b]; });
    int *ts = host_ints.data();
    int *tm = ts + (size_t)ns * nr;
    int *ts64 = tm + ns;
    int *tm64 = ts64 + (size_t)ns * nr64;
    int *ls = tm64 + ns;
    int *sm = ls + ns;
    int *cnt = sm + ns;
    auto build = [&](int *tsl, int *tms, int tile) {
        std::fill(tsl, tsl + (size_t)ns * tile, -1);
        std::fill(tms, tms + ns, 0);
        int nt = 0;
        for (size_t i = 0; i < sorted.size();) {
            const int m = mass[sorted[i]];
            int k = 0;
            while (k < tile && i < sorted.size() && mass[sorted[i]] == m) tsl[(size_t)nt * tile + k++] = sorted[i++];
            tms[nt++] = m;
        }
        return nt;
    };
    cnt[0] = build(ts, tm, nr);
    cnt[2] = build(ts64, tm64, nr64);
    if (cnt[0] > tiles_cap || cnt[2] > tiles64_cap)
        return set_error(LAPH_ERR_INVALID, "slot masses outside the context's mass table");
    for (size_t i = 0; i < slots.size(); ++i) ls[i] = slots[i];
    for (int s = 0; s < ns; ++s) sm[s] = s < (int)mass.size() ? mass[s] : 0;
    cnt[1] = (int)slots.size();
    LAPH_HIP(hipMemcpyAsync(ws.tile_slots, host_ints.data(), host_ints.size() * sizeof(int), hipMemcpyHostToDevice,
                            c->stream));
    // the copy reads host_ints asynchronously: wait before the buffer can change
    LAPH_HIP(hipStreamSynchronize(c->stream));
    return LAPH_OK;
}

laph_status Solver::download_state() {
    LAPH_HIP(hipMemcpyAsync(host_st.data(), ws.st, ns * sizeof(SlotState), hipMemcpyDeviceToHost, c->stream));
    LAPH_HIP(hipStreamSynchronize(c->stream));
    return LAPH_OK;
}

laph_status Solver::upload_state() {
    LAPH_HIP(hipMemcpyAsync(ws.st, host_st.data(), ns * sizeof(SlotState), hipMemcpyHostToDevice, c->stream));
    LAPH_HIP(hipStreamSynchronize(c->stream));
    return LAPH_OK;
}

// ---- stencil helpers --------------------------------------------------------
// workgroups of a flagged (reliable-update) stage launch: a few per CU
constexpr int kFlaggedGrid = 2048;

laph_status Solver::stage(int sprec, int out_parity, Operand in, Operand out, int clover, int pre, Operand z,
                          double cz, int post, Operand y, double a, Operand y2, double a2, double b, int red,
                          Operand w, int flagged, SiteWindow win) {
    StageSpec s;
    s.prec = sprec;
    s.out_parity = out_parity;
    s.dagger = p.dagger;
    s.clover = clover;
    s.pre = pre;
    s.post = post;
    s.red = red;
    s.flagged = flagged;
    s.in = in;
    s.out = out;
    s.y = y;
    s.y2 = y2;
    s.z = z;
    s.w = w;
    s.a = a;
    s.a2 = a2;
    s.b = b;
    s.c = cz;
    const bool f64 = sprec == LAPH_F64;
    s.tiles = tiles(f64, flagged != 0);
    s.form = f64 ? form64 : form;
    s.site_major = f64 ? site_major64 : site_major;
    // the flagged count is known only on the device: a small grid walks the live tiles
    s.grid_cap = flagged ? kFlaggedGrid : 0;
    s.slots = ws.st;
    s.partials = ws.partials;
    s.pstride = pstride;
    s.win = win;
    return launch_stage(*c, s);
}

laph_status Solver::clover(int parity, int inverse, Operand in, Operand out, int post, Operand y, double a, double b,
                           int nlist, SiteWindow win) {
    CloverSpec s;
    s.prec = LAPH_F64;
    s.parity = parity;
    s.inverse = inverse;
    s.post = post;
    s.in = in;
    s.out = out;
    s.y = y;
    s.a = a;
    s.b = b;
    s.slot_list = ws.list;
    s.slot_mass = ws.slot_mass;
    s.n = nlist;
    s.win = win;
    return launch_clover(*c, s);
}

// ---- one BiCGStab iteration (all kernels device-driven) ---------------------
laph_status Solver::iteration() {
    const Operand none;
    BlasArgs a = blas(ns);
    FinArgs f = fin(ns);
    LAPH_TRY(blas_p_update(*c, a, prec));
    // v = M_hat p,  <r^, v>
    LAPH_TRY(stage(prec, 1, ws.p, ws.tmp, 1, 0, none, 0, 0, none, 0, none, 0, 1.0, 0, none, 0));
    LAPH_TRY(stage(prec, 0, ws.tmp, ws.v, 1, 0, none, 0, 1, ws.p, 1.0, none, 0, -0.25, 1, ws.rh, 0));
    LAPH_TRY(blas_finalize(*c, fin(ns, nsb_inner), kFinAlpha));
    // s = r - alpha v (in r)
    LAPH_TRY(blas_s_update(*c, a, prec));
    // t = M_hat s,  <t, s>, |t|^2
    LAPH_TRY(stage(prec, 1, ws.r, ws.tmp, 1, 0, none, 0, 0, none, 0, none, 0, 1.0, 0, none, 0));
    LAPH_TRY(stage(prec, 0, ws.tmp, ws.t, 1, 0, none, 0, 1, ws.r, 1.0, none, 0, -0.25, 2, none, 0));
    LAPH_TRY(blas_finalize(*c, fin(ns, nsb_inner), kFinOmega));
    // x_lo += alpha p + omega s;  r = s - omega t;  rho, |r|^2, update decision
    LAPH_TRY(blas_xr_update(*c, a, prec));
    LAPH_TRY(blas_finalize(*c, f, kFinRho));
    // compact the slots flagged for a reliable update (list and FP64 tiles)
    FlagArgs fl;
    fl.tile_slots = ws.tile64_slots;
    fl.tile_mass = ws.tile64_mass;
    fl.ntiles = ws.ntiles64;
    fl.nr = nr64;
    fl.st = ws.st;
    fl.out_slots = ws.tile64f_slots;
    fl.out_mass = ws.tile64f_mass;
    fl.out_ntiles = ws.ntiles64f;
    fl.flist = ws.flist;
    fl.nflist = ws.nflist;
    LAPH_TRY(blas_flag_tiles(*c, fl));
    // reliable update of the flagged slots: x64 += x_lo and the FP64 residual of x64.
    // With an FP32 x_lo and the LDS form the residual follows the same exact correction,
    // r64 -= M_hat x_lo in FP64 arithmetic on the widened x_lo (the stages read x_lo, half
    // the bytes of x64, and r64 in place of b_hat), and the second stage also folds x_lo
    // into x64 (x_lo of a flagged slot is never marked zero here: every iteration's x/r
    // update writes it before the update decision); otherwise x64 += x_lo, then
    // r64 = b_hat - M_hat x64
    if (prec != LAPH_F64 && form64 == kFormLds) {
        LAPH_TRY(stage(LAPH_F64, 1, ws.x, ws.O0, 1, 0, none, 0, 0, none, 0, none, 0, 1.0, 6, none, 1));
        LAPH_TRY(stage(LAPH_F64, 0, ws.O0, ws.E2, 1, 0, none, 0, 2, ws.E2, 1.0, ws.x, -1.0, 0.25, 7, ws.E1, 1));
    } else {
        LAPH_TRY(blas_accumulate(*c, a, prec, kModeFlagged));
        LAPH_TRY(stage(LAPH_F64, 1, ws.E1, ws.O0, 1, 0, none, 0, 0, none, 0, none, 0, 1.0, 0, none, 1));
        LAPH_TRY(stage(LAPH_F64, 0, ws.O0, ws.E2, 1, 0, none, 0, 2, ws.E0, 1.0, ws.E1, -1.0, 0.25, 3, none, 1));
    }
    LAPH_TRY(blas_finalize(*c, fin(ns, nsb64), kFinUpdate));
    LAPH_TRY(blas_lower(*c, a, prec, kModeFlagged, 0));
    LAPH_TRY(blas_finalize(*c, f, kFinRho2));
    return LAPH_OK;
}

laph_status Solver::run_iterations(int k) {
    if (!p.use_graph) {
        for (int i = 0; i < k; ++i) LAPH_TRY(iteration());
        return LAPH_OK;
    }
    if (!graph_exec || graph_k != k) {
        if (graph_exec) {
            (void)hipGraphExecDestroy(graph_exec);
            graph_exec = nullptr;
        }
        hipGraph_t graph = nullptr;
        LAPH_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
        laph_status st = LAPH_OK;
        for (int i = 0; i < k && st == LAPH_OK; ++i) st = iteration();
        hipError_t e = hipStreamEndCapture(c->stream, &graph);
        if (st != LAPH_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return set_error(LAPH_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&graph_exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            graph_exec = nullptr;
            return set_error(LAPH_ERR_HIP, "graph instantiate failed: %s", hipGetErrorString(e));
        }
        graph_k = k;
    }
    LAPH_HIP(hipGraphLaunch(graph_exec, c->stream));
    return LAPH_OK;
}

// ---- sources ------------------------------------------------------------------
laph_status Solver::load_sources(const SourceSpec &src) {
    if (src.B) {
        Operand e = ws.E0, o = ws.O1;
        LAPH_TRY(pack_spinor(*c, e, src.B, LAPH_F64, src.n, 0, src.B_stride));
        LAPH_TRY(pack_spinor(*c, o, src.B, LAPH_F64, src.n, 1, src.B_stride));
        return LAPH_OK;
    }
    return make_laph_sources(*c, ws.E0, ws.O1, src.V, src.nev, src.t0, src.r_begin, src.n, src.rho, src.n_dil);
}

// b_e into E0 (sites outside win are left as they are)
laph_status Solver::load_even_source(const SourceSpec &src, SiteWindow win) {
    if (src.B) return pack_spinor(*c, ws.E0, src.B, LAPH_F64, src.n, 0, src.B_stride);
    return make_laph_sources(*c, ws.E0, ws.O1, src.V, src.nev, src.t0, src.r_begin, src.n, src.rho, src.n_dil, 0,
                             win);
}

// ---- the full solve of n slots ----------------------------------------------------
laph_status Solver::solve(const SourceSpec &src, const std::vector<int> &slot_mass, double tol, const double *X0,
                          size_t X0_stride) {
    const int n = src.n;
    if (n > ns) return set_error(LAPH_ERR_INVALID, "batch larger than the workspace");
    mass = slot_mass;
    const Operand none;
    std::vector<int> all(n);
    for (int i = 0; i < n; ++i) all[i] = i;
    LAPH_TRY(upload_tables(all));
    double delta = p.delta;
    // defaults measured on the 32^3 x 64 perambulator: delta 0.1 / 0.02 / 0.01 / 0.005 /
    // 0.002 gave 8.8 / 5.9 / 5.0 / 4.45 / 4.0 FP64 updates per RHS at 29.0 / 29.2 / 29.4 /
    // 29.7 / 30.2 iterations (FP16N inner); FP32 inner kept its iteration count down to
    // 0.001 (3.9 updates)
    if (delta <= 0) delta = prec == LAPH_F16N ? 0.005 : (prec == LAPH_F32 ? 0.001 : 0.0);
    const int maxiter = p.maxiter > 0 ? p.maxiter : 10000;
    for (int s = 0; s < ns; ++s) {
        SlotState z{};
        z.status = s < n ? LAPH_RHS_ACTIVE : LAPH_RHS_CONVERGED;
        z.delta2 = delta * delta;
        z.maxiter = maxiter;
        host_st[s] = z;
    }
    LAPH_TRY(upload_state());
    BlasArgs a = blas(n);
    FinArgs f = fin(n);
    // LapH and noise sources live on timeslice t0 alone, so the source preparation
    // touches only a slab around it: A_oo^-1 b_o is computed on t0 +- 2 (the slices the
    // next stage reads; zero but for t0), b_hat on t0 +- 1 (E0 keeps the zeros the
    // sources put elsewhere), and |B|^2 and the copy r64 = b_hat read only those slices
    const bool slab = src.B == nullptr && src.V != nullptr;
    const SiteWindow w_src = slab ? slab_window(c->g, src.t0, 0) : SiteWindow();
    const SiteWindow w_hat = slab ? slab_window(c->g, src.t0, 1) : SiteWindow();
    const SiteWindow w_clv = slab ? slab_window(c->g, src.t0, 2) : SiteWindow();
    // |B|^2 and the stopping threshold on the even-odd residual
    LAPH_TRY(load_sources(src));
    BlasArgs a_src = a;
    a_src.win = w_src;
    LAPH_TRY(blas_norm2(*c, a_src, ws.E0, ws.O1, kModeAll));
    LAPH_TRY(blas_finalize(*c, f, kFinBnorm));
    LAPH_TRY(download_state());
    // |B - D X| = |A_ee r_e| for an exactly reconstructed odd half; 0.2 covers |A_ee| <~ 5
    double stop_fac = 0.2 * tol;
    for (int s = 0; s < n; ++s) {
        SlotState &st = host_st[s];
        st.stop2 = stop_fac * stop_fac * st.bnorm2;
        if (st.status == LAPH_RHS_ACTIVE && st.bnorm2 == 0.0) st.status = LAPH_RHS_CONVERGED;
    }
    LAPH_TRY(upload_state());
    bool have_x = X0 != nullptr;
    if (have_x) LAPH_TRY(pack_spinor(*c, ws.E1, X0, LAPH_F64, n, 0, X0_stride));
    else LAPH_HIP(hipMemsetAsync(ws.E1.base, 0, ws.E1.stride * n, c->stream));

    // slots the current pass works on (all of them first, then those that missed tol)
    std::vector<int> cur = all;
    for (int pass = 0; pass < 4; ++pass) {
        const int ncur = (int)cur.size();
        a = blas(ncur);
        f = fin(ncur);
        // prepared source b_hat = A_ee^-1 (b_e + 1/2 H_eo A_oo^-1 b_o) in E0 (O0 scratch)
        LAPH_TRY(clover(1, 1, ws.O1, ws.O0, 0, none, 0, 1.0, ncur, w_clv));
        LAPH_TRY(stage(LAPH_F64, 0, ws.O0, ws.E0, 1, 1, ws.E0, 2.0, 0, none, 0, none, 0, 0.5, 0, none, 0, w_hat));
        // r64 = b_hat - M_hat x64
        if (have_x) {
            LAPH_TRY(stage(LAPH_F64, 1, ws.E1, ws.O0, 1, 0, none, 0, 0, none, 0, none, 0, 1.0, 0, none, 0));
            LAPH_TRY(stage(LAPH_F64, 0, ws.O0, ws.E2, 1, 0, none, 0, 2, ws.E0, 1.0, ws.E1, -1.0, 0.25, 3, none, 0));
        } else {
            BlasArgs a_hat = a;
            a_hat.win = w_hat;
            LAPH_TRY(blas_copy64(*c, a_hat, ws.E2, ws.E0, kModeActive));
            LAPH_TRY(blas_norm2(*c, a_hat, ws.E2, none, kModeActive));
        }
        // partials of the FP64 stage (warm start) or of the norm kernel
        LAPH_TRY(blas_finalize(*c, have_x ? fin(ncur, nsb64) : f, kFinR64));
        LAPH_TRY(blas_lower(*c, a, prec, kModeActive, 1));
        LAPH_TRY(blas_finalize(*c, f, kFinInit));
        // iterate; the captured graph always spans ns slots (tables say which are live)
        LAPH_TRY(download_state());
        std::vector<int> active;
        for (int s : cur)
            if (host_st[s].status == LAPH_RHS_ACTIVE) active.push_back(s);
        LAPH_TRY(upload_tables(active));
        const int K = p.graph_iters > 0 ? p.graph_iters : 8;
        int guard = 0;
        while (!active.empty()) {
            LAPH_TRY(run_iterations(K));
            LAPH_TRY(download_state());
            std::vector<int> still;
            for (int s : active)
                if (host_st[s].status == LAPH_RHS_ACTIVE) still.push_back(s);
            if (still.size() != active.size()) {
                active.swap(still);
                if (!active.empty()) LAPH_TRY(upload_tables(active));
            }
            if (++guard * K > maxiter + 4 * K) break;
        }
        // all slots of the batch from here on
        LAPH_TRY(upload_tables(all));
        a = blas(n);
        f = fin(n);
        // any slot still active (host guard): fold x_lo into x64
        LAPH_TRY(blas_accumulate(*c, a, prec, kModeActive));
        // reconstruct x_o = A_oo^-1 v, v = b_o + 1/2 H_oe x_e, into O0, and the true
        // residual |B - D X|^2.  Its odd part is |v - A_oo x_o|^2: the LDS form takes it in
        // the reconstructing pass (b_o stays in O1) and the even part in one more stage;
        // otherwise each part is built by a clover pass and a stage
        const bool fused_odd = form64 == kFormLds;
        if (!fused_odd)
            LAPH_TRY(stage(LAPH_F64, 1, ws.E1, ws.O0, 1, 1, ws.O1, 2.0, 0, none, 0, none, 0, 0.5, 0, none, 0));
        LAPH_TRY(download_state());
        for (int s = 0; s < n; ++s) host_st[s].true_res2 = 0;
        LAPH_TRY(upload_state());
        if (fused_odd) {
            LAPH_TRY(stage(LAPH_F64, 1, ws.E1, ws.O0, 1, 1, ws.O1, 2.0, 0, none, 0, none, 0, 0.5, 4, none, 0));
            LAPH_TRY(blas_finalize(*c, fin(n, nsb64), kFinTrueRes));
        }
        // even part in E0: b_e again (E0 held b_hat, which LapH sources leave zero outside
        // t0 +- 1), b_e - A_ee x_e + 1/2 H_eo x_o
        LAPH_TRY(load_even_source(src, w_hat));
        if (fused_odd) {
            // one pass: b_e + 1/2 H_eo x_o - A_ee x_e
            LAPH_TRY(stage(LAPH_F64, 0, ws.O0, ws.E0, 0, 0, none, 0, 2, ws.E0, 1.0, ws.E1, 0, 0.5, 5, none, 0));
        } else {
            LAPH_TRY(clover(0, 0, ws.E1, ws.E0, 1, ws.E0, 1.0, -1.0, n));
            LAPH_TRY(stage(LAPH_F64, 0, ws.O0, ws.E0, 0, 0, none, 0, 1, ws.E0, 1.0, none, 0, 0.5, 3, none, 0));
        }
        LAPH_TRY(blas_finalize(*c, fin(n, nsb64), kFinTrueRes));
        if (!fused_odd) {
            LAPH_TRY(clover(1, 0, ws.O0, ws.O1, 1, ws.O1, 1.0, -1.0, n));
            LAPH_TRY(stage(LAPH_F64, 1, ws.E1, ws.O1, 0, 0, none, 0, 1, ws.O1, 1.0, none, 0, 0.5, 3, none, 0));
            LAPH_TRY(blas_finalize(*c, fin(n, nsb64), kFinTrueRes));
        }
        LAPH_TRY(download_state());
        // slots that converged on the even-odd residual but miss tol on the full one go again
        std::vector<int> redo;
        for (int s = 0; s < n; ++s) {
            SlotState &st = host_st[s];
            const double tr = st.bnorm2 > 0 ? std::sqrt(st.true_res2 / st.bnorm2) : 0.0;
            if (st.status == LAPH_RHS_CONVERGED && tr > tol && st.bnorm2 > 0) redo.push_back(s);
        }
        if (redo.empty() || pass == 3) break;
        for (int s : redo) {
            SlotState &st = host_st[s];
            const double tr = std::sqrt(st.true_res2 / st.bnorm2);
            st.stop2 *= 0.25 * (tol / tr) * (tol / tr);
            st.status = LAPH_RHS_ACTIVE;
            st.flag = 0;
        }
        LAPH_TRY(upload_state());
        LAPH_TRY(upload_tables(redo));
        cur = redo;
        // sources again (E0 and O1 were overwritten by the residual check)
        LAPH_TRY(load_sources(src));
        have_x = true;
    }
    return LAPH_OK;
}

laph_status Solver::collect(laph_rhs_stats *out, int n, double tol, int *worst) {
    LAPH_TRY(download_state());
    int w = LAPH_OK;
    for (int s = 0; s < n; ++s) {
        const SlotState &st = host_st[s];
        const double tr = st.bnorm2 > 0 ? std::sqrt(st.true_res2 / st.bnorm2) : 0.0;
        int status = st.status;
        if (status == LAPH_RHS_CONVERGED && !(tr <= tol)) status = LAPH_RHS_NOCONV;
        if (status == LAPH_RHS_ACTIVE) status = LAPH_RHS_NOCONV;
        if (!std::isfinite(tr)) status = LAPH_RHS_NONFINITE;
        if (out) {
            out[s].status = status;
            out[s].iters = st.iters;
            out[s].updates = st.updates;
            out[s].restarts = st.restarts;
            out[s].true_res = tr;
        }
        int code = status == LAPH_RHS_CONVERGED ? LAPH_OK
                   : status == LAPH_RHS_NONFINITE ? LAPH_ERR_NONFINITE
                   : status == LAPH_RHS_BREAKDOWN ? LAPH_ERR_BREAKDOWN
                                                  : LAPH_ERR_NOCONV;
        if (code == LAPH_ERR_NONFINITE || (code == LAPH_ERR_BREAKDOWN && w != LAPH_ERR_NONFINITE) ||
            (code == LAPH_ERR_NOCONV && w == LAPH_OK))
            w = code;
    }
    *worst = w;
    return LAPH_OK;
}

}  // namespace laph
