// The batched mixed-precision BiCGStab driver (solver.hip) and the LapH
// source / projection kernels it feeds (project.hip).
#pragma once

#include <vector>

#include "laph_blas.h"

namespace laph {

// Where the right-hand sides come from: canonical sources B (slot s = RHS s,
// B + s * B_stride doubles... in complex128 elements), or spin-diluted LapH
// sources r_begin .. r_begin + n - 1 built from V at t0.
struct SourceSpec {
    const double *B = nullptr;
    size_t B_stride = 0;   // complex elements between RHS (0: one full lattice)
    const double *V = nullptr;
    int nev = 0, t0 = 0, r_begin = 0;
    int n = 0;
    const double *rho = nullptr;   // noise [4][nev] complex (null: the perambulator's sources)
    int n_dil = 0;
};

// b^(r)(x, t)_(s, a) = delta_{t,t0} delta_{s,alpha} V_k(x, t0)_a, r = 4k + alpha, for
// r = r_begin .. r_begin + n - 1, into FP64 even (E) and odd (O) half-vectors; with
// noise rho, r = 4j + alpha and V_k becomes sum_{k = j mod n_dil} rho[alpha][k] V_k.
// parity 0 / 1: that half only; sites outside win are not written.
laph_status make_laph_sources(const Ctx &c, Operand E, Operand O, const double *V, int nev, int t0, int r_begin,
                              int n, const double *rho = nullptr, int n_dil = 0, int parity = -1,
                              SiteWindow win = SiteWindow());

// Projection of FP64 internal solutions onto the LapH vectors of every sink
// timeslice, accumulated into tau[t][l][k][beta][alpha] for RHS r = r_begin + s.
struct ProjectSpec {
    Operand xe, xo;           // FP64 internal even / odd halves, slot s = RHS r_begin + s
    int n = 0;                // RHS in this batch
    int r_begin = 0;
    const double *Vp = nullptr;   // V packed to the internal site order (pack_laph_vectors)
    int nev = 0;                  // sink vectors
    int nev_src = 0;              // source vectors (tau's k extent)
    double *tau = nullptr;
    double *scratch = nullptr;    // project_scratch_bytes
};
size_t packed_v_bytes(const Ctx &c, int nev);
laph_status pack_laph_vectors(const Ctx &c, double *Vp, const double *V, int nev);
size_t project_scratch_bytes(const Ctx &c, int nev, int n);
laph_status project(const Ctx &c, const ProjectSpec &s);
laph_status project_adjoint(const Ctx &c, double *GX, const double *Gtau, const double *V, int nev, int nev_src);
// tau' = S tau S^dagger on nblk consecutive 4 x 4 complex blocks (S: host, row-major)
laph_status spin_rotate(const Ctx &c, double *out, const double *tau, long nblk, const double *S_host);
laph_status make_sources_canonical(const Ctx &c, double *B, const double *V, int nev, int t0,
                                   const double *rho = nullptr, int n_dil = 0);

// LapH eigenvectors (laplace.hip): out[t][j] = (-Delta) in[t][j] per timeslice, and the
// lowest nev eigenpairs of -Delta on every timeslice (Chebyshev-filtered subspace
// iteration; V[t][l][z][y][x][a], lambda_host[t][l] ascending).
laph_status apply_neg_laplacian(const Ctx &c, double *out, const double *in, int nvec);
size_t laplacian_eig_workspace_bytes(const Ctx &c, int nev);
laph_status laplacian_eigvecs(Ctx &c, double *V, double *lambda_host, int nev, double tol, int max_iter, int degree,
                              char *work, size_t bytes, int *iters_out, double *res_host);

// Meson doublets (kind 0) and baryon triplets (kind 1) of the LapH vectors per
// timeslice and momentum (contract.hip).
size_t contract_workspace_bytes(const Ctx &c, int kind, int nev, int n_mom);
laph_status contract(const Ctx &c, int kind, double *out, const double *V, int nev, int n_mom, const int *mom_host,
                     char *work, size_t bytes);

class Solver {
   public:
    struct WS {
        Operand E0, E1, E2, O0, O1;        // FP64 halves: b_hat/b_e, x64, r64, x_o/scratch, b_o
        Operand r, rh, p, v, t, tmp, x;    // inner precision; x in the x_lo precision
        SlotState *st = nullptr;
        double *partials = nullptr;
        int *tile_slots = nullptr, *tile_mass = nullptr;      // inner-form tiles
        int *tile64_slots = nullptr, *tile64_mass = nullptr;  // FP64 register tiles
        int *tile64f_slots = nullptr, *tile64f_mass = nullptr;  // FP64 tiles of the flagged slots
        int *list = nullptr, *slot_mass = nullptr, *flist = nullptr;
        int *ntiles = nullptr, *nlist = nullptr, *ntiles64 = nullptr, *ntiles64f = nullptr, *nflist = nullptr;
        int *ints = nullptr;          // integer region the tables are carved from
        size_t nints = 0, nints_used = 0;
    };

    static void choose_shape(const laph_solve_params &p, int ns, int &form, int &nr, int &form64, int &nr64);
    static size_t layout(const Ctx &c, int ns, int prec, char *base, WS *ws);
    // tune_mass >= 0: with stencil == 0 and rhs_tile <= 0, measure the stencil shape
    // for this batch if no tuned choice exists yet (on the workspace, before use)
    laph_status init(Ctx &ctx, int nslots, const laph_solve_params &params, char *work, size_t bytes,
                     int tune_mass = -1);
    ~Solver();

    // Solve the n = src.n RHS of one batch (slot s <- RHS s of the spec).
    laph_status solve(const SourceSpec &src, const std::vector<int> &slot_mass, double tol, const double *X0,
                      size_t X0_stride);
    laph_status collect(laph_rhs_stats *out, int n, double tol, int *worst);
    const WS &workspace() const { return ws; }

   private:
    const Ctx *c = nullptr;
    laph_solve_params p{};
    int ns = 0, prec = 0, form = kFormRegister, nr = 1, nr64 = 1, site_major = 0, nsb256 = 0, nsb_inner = 0,
        pstride = 0;
    int form64 = kFormRegister, site_major64 = 0, nsb64 = 0;   // shape of the FP64 stages
    // most tiles a table can hold (tiles never mix masses): the launch grids
    int tiles_cap = 0, tiles64_cap = 0;
    WS ws;
    std::vector<int> mass;
    std::vector<int> host_ints;
    std::vector<SlotState> host_st;
    hipGraphExec_t graph_exec = nullptr;
    int graph_k = 0;

    void carve_tables();
    BlasArgs blas(int list_max) const;
    FinArgs fin(int list_max, int nsb = 0) const;
    Tiles tiles(bool f64, bool flagged = false) const;
    laph_status upload_tables(const std::vector<int> &slots);
    laph_status download_state();
    laph_status upload_state();
    laph_status stage(int sprec, int out_parity, Operand in, Operand out, int clover, int pre, Operand z, double cz,
                      int post, Operand y, double a, Operand y2, double a2, double b, int red, Operand w, int flagged,
                      SiteWindow win = SiteWindow());
    laph_status clover(int parity, int inverse, Operand in, Operand out, int post, Operand y, double a, double b,
                       int nlist, SiteWindow win = SiteWindow());
    laph_status iteration();
    laph_status run_iterations(int k);
    laph_status load_sources(const SourceSpec &src);
    laph_status load_even_source(const SourceSpec &src, SiteWindow win);
};

}  // namespace laph
