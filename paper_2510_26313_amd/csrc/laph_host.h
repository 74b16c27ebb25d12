// Host-side context and launcher declarations of liblaph.
#pragma once

#include <map>
#include <string>
#include <utility>
#include <vector>

#include "laph_internal.h"

namespace laph {

// A right-hand-side operand: the half-vector of slot s starts at base + s * stride.
struct Operand {
    char *base = nullptr;
    size_t stride = 0;
    __host__ __device__ char *at(int s) const { return base + (size_t)s * stride; }
};

// Device-resident per-slot solver state (one per right-hand side in a batch).
struct SlotState {
    double2 rho, rho_prev, alpha, omega, beta;
    double r2;        // |r_inner|^2
    double r2_upd;    // |r64|^2 at the last reliable update
    double stop2;     // stop when |r64|^2 <= stop2 (even-odd system)
    double bnorm2;    // |B|^2 of the full-lattice source
    double delta2;    // reliable-update trigger (delta^2)
    double true_res2; // |B - D X|^2 / |B|^2 at exit
    int status;       // LAPH_RHS_*
    int flag;         // 1: reliable update requested, 2: update + restart (breakdown)
    int iters, updates, restarts, maxiter;
    int xlo_zero;     // 1: x_lo is zero (its memory is stale and not read) until the next x/r update
};

// Two forms of the stencil stage kernel: RHS tiles held in registers by one
// thread, or RHS-parallel waves sharing links staged in LDS.
enum { kFormRegister = 0, kFormLds = 1 };

// Tile table shared by the stencil kernels: tile j holds up to nr slots of one mass.
struct Tiles {
    const int *slots = nullptr;   // [ntiles_max][nr], -1 = empty
    const int *mass = nullptr;    // [ntiles_max]
    const int *ntiles = nullptr;  // device scalar: active tiles
    int ntiles_max = 0;
    int nr = 1;
};

// Two-level aggregation multigrid attached to a context (mg.hip): geometry of
// the aggregates and the device arrays inside the caller's multigrid buffer.
struct MgGeom {
    int block[4] = {0, 0, 0, 0};   // aggregate extents (x, y, z, t)
    int cdim[4] = {0, 0, 0, 0};    // coarse lattice extents
    int nc = 0;                    // coarse sites
    int asize = 0;                 // fine sites per aggregate
    int nv = 0;                    // near-null vectors
    int ncv = 0;                   // coarse components per coarse site (2 nv)
};
struct MgState {
    bool ready = false;
    int mass_idx = 0;
    MgGeom geo;
    int smooth_iters = 4, coarse_iters = 16, restart = 8, maxiter = 200;
    double coarse_tol = 0.1;
    char *basis = nullptr;        // nv full FP64 fields (even half, odd half)
    size_t basis_stride = 0;      // bytes per field
    char *basis32 = nullptr;      // the same in FP32 (the cycle's restriction and prolongation)
    size_t basis32_stride = 0;
    double2 *coarse = nullptr;    // [nc][9][ncv][ncv]
    int *flag = nullptr;          // device int: set by a failed setup step
};

struct Ctx {
    Geom g{};
    int dims[4]{};
    int n_mass_max = 0;
    hipStream_t stream = nullptr;
    int device = -1;   // HIP device current at laph_create (-1: none)
    char *state = nullptr;
    size_t state_size = 0;
    // offsets inside the state buffer
    size_t off_g64 = 0, off_g32 = 0, off_g16a = 0, off_g16b = 0, off_clov = 0, off_misc = 0, off_inv64 = 0,
           off_inv32 = 0;
    size_t sz_g64_pm = 0, sz_g32_pm = 0, sz_g16a_pm = 0, sz_g16b_pm = 0;   // per (parity, mu)
    size_t sz_cl64_par = 0, sz_cl32_par = 0;                              // per parity
    bool gauge_loaded = false;
    int n_mass = 0;
    double csw = 0;
    std::vector<double> m0;
    GaugePtrs gp{};
    // small pinned host buffers for polling and tile uploads
    int *pinned_i = nullptr;
    size_t pinned_i_len = 0;
    hipEvent_t ev[4]{};
    double last_ms[3]{};
    // device architecture (gcnArchName up to the first ':'), the autotune cache key
    char arch[64] = "unknown";
    // autotuned stencil shape per (inner precision, batch size)
    struct Shape {
        int form, tile, site_major;
    };
    std::map<std::pair<int, int>, Shape> tuned;
    MgState mgs;   // the attached multigrid (laph_mg_setup)

    size_t hv(int prec) const { return hv_bytes(prec, (size_t)g.vh); }
    // misc region: per-mass diagonal 4 + m0, the SU(3) deviation and the clover failure flag
    double *mass_diag() const { return reinterpret_cast<double *>(state + off_misc); }
    unsigned long long *gauge_dev() const {
        return reinterpret_cast<unsigned long long *>(state + off_misc + round256(8 * (size_t)n_mass_max));
    }
    int *bad_flag() const { return reinterpret_cast<int *>(state + off_misc + round256(8 * (size_t)n_mass_max) + 64); }
    // clover data of a parity: term (FP64), inverse of mass m (FP64 / FP32)
    const char *clover_term(int parity) const { return state + off_clov + parity * sz_cl64_par; }
    const char *clover_inv64(int mass, int parity) const {
        return state + off_inv64 + ((size_t)mass * 2 + parity) * sz_cl64_par;
    }
    const char *clover_inv32(int mass, int parity) const {
        return state + off_inv32 + ((size_t)mass * 2 + parity) * sz_cl32_par;
    }
    size_t clover_inv_mass_stride(int prec) const { return 2 * (prec == LAPH_F64 ? sz_cl64_par : sz_cl32_par); }
    const char *clover_inv(int prec, int mass, int parity) const {
        return prec == LAPH_F64 ? clover_inv64(mass, parity) : clover_inv32(mass, parity);
    }
};

// ---- error handling ----------------------------------------------------------
laph_status set_error(laph_status st, const char *fmt, ...);
#define LAPH_HIP(call)                                                                          \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return ::laph::set_error(LAPH_ERR_HIP, "%s failed: %s (%s:%d)", #call,               \
                                     hipGetErrorString(e_), __FILE__, __LINE__);                \
    } while (0)
#define LAPH_TRY(expr)                 \
    do {                               \
        laph_status s_ = (expr);       \
        if (s_ != LAPH_OK) return s_;  \
    } while (0)
laph_status check_launch(const char *what);

// ---- stencil stages (dslash.hip) ---------------------------------------------
// out = a*y + a2*y2 + b * [A^-1] (c*z + H_{p,1-p} in)   per slot of every tile,
// with optional fused FP64 reductions written as per-block partials:
//   red 0: none; 1: <w, out> (2 doubles); 2: <out, y>, |out|^2 (3 doubles); 3: |out|^2 (1 double)
struct StageSpec {
    int prec = LAPH_F64;
    int out_parity = 0;
    int dagger = 0;
    int clover = 0;   // apply A^-1 of the output parity (mass from the tile)
    int pre = 0;      // c*z inside the clover
    int post = 0;     // number of post terms (0, 1, 2)
    int red = 0;
    int flagged = 0;  // only slots whose SlotState.flag != 0 (and status active)
    Operand in, out, y, y2, z, w;
    double a = 0, a2 = 0, b = 1, c = 0;
    Tiles tiles;
    int site_major = 0;                 // 1: each tile sweeps all site blocks (see stage_item)
    int grid_cap = 0;                   // > 0: at most this many workgroups, each walking several items
    int form = kFormRegister;           // kFormRegister: tiles.nr RHS per thread;
                                        // kFormLds: tiles.nr = 4 * RW RHS per workgroup, links in LDS
    const SlotState *slots = nullptr;   // may be null when flagged == 0
    double *partials = nullptr;         // [slot][3][pstride]
    int pstride = 0;                    // partials per quantity per slot (>= stage_nsb)
    SiteWindow win;                     // output sites computed (the others untouched); red == 0 only
};
// site blocks of a stage launch (= partial sums it writes per quantity and slot)
int stage_nsb(const Ctx &c, int form);
// a partial-sum stride large enough for every kernel of the library
int partial_stride(const Ctx &c);
laph_status launch_stage(const Ctx &c, const StageSpec &s);

// out = a*y + b * M in with M = A (inverse = 0) or A^-1 of the given parity,
// per slot in a slot list.
struct CloverSpec {
    int prec = LAPH_F64;
    int parity = 0;
    int inverse = 1;
    int post = 0;
    Operand in, out, y;
    double a = 0, b = 1;
    const int *slot_list = nullptr;   // [n] slots (null: identity slot = index)
    const int *slot_mass = nullptr;   // [slot] mass index (null: mass_idx for all)
    int mass_idx = 0;
    int n = 0;
    SiteWindow win;                   // sites computed (the others untouched)
};
laph_status launch_clover(const Ctx &c, const CloverSpec &s);

// ---- autotuner (tune.hip) ------------------------------------------------------
// Time the solver's two fused stages for nrhs RHS in one form / tile; fields holds
// 4 * nrhs half-vectors of prec, partials nrhs * 3 * partial_stride doubles,
// d_ints tune_ints(nrhs) ints.
laph_status time_stage_pair(const Ctx &c, int prec, int nrhs, int form, int tile, int site_major, int mass_idx,
                            int reps, char *fields, double *partials, int *d_ints, double ms[2]);
laph_status autotune_stencil(Ctx &c, int prec, int nrhs, int mass_idx, char *fields, double *partials, int *d_ints,
                             Ctx::Shape *out, double *ms_out);
void load_tune_cache(Ctx &c);
size_t tune_ints(int nrhs);

// ---- setup kernels (setup.hip) ------------------------------------------------
laph_status load_gauge(Ctx &c, const double *U);
laph_status build_clover(Ctx &c, double csw, int n_mass, const double *m0);
laph_status pack_spinor(const Ctx &c, Operand out, const double *in, int prec, int nrhs, int parity,
                        size_t in_rhs_stride_elems = 0);
laph_status unpack_spinor(const Ctx &c, double *out, Operand in, int prec, int nrhs, int parity,
                          size_t out_rhs_stride_elems = 0);

// ---- solver (solver.hip) --------------------------------------------------------
struct SolveJob {
    // canonical inputs / outputs (either B or V-sources)
    const double *B = nullptr;     // canonical sources, or null when sources come from V
    const double *V = nullptr;     // LapH vectors (sources built at t0)
    int t0 = 0, nev = 0, k_begin = 0;
    int nrhs = 0;
    std::vector<int> mass;         // per RHS
    double tol = 1e-10;
    laph_solve_params p{};
};
size_t solver_workspace_bytes(const Ctx &c, int nslots, const laph_solve_params &p);

}  // namespace laph
