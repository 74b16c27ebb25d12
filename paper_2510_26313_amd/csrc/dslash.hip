// Launch of the even-odd stencil stages (kernels in dslash_kernels.h) and the
// single-parity clover apply kernel.
#include "dslash_lds.h"

namespace laph {

int stage_nsb(const Ctx &c, int form) {
    const int sites = form == kFormLds ? kLdsSites : kBlock;
    return (c.g.vh + sites - 1) / sites;
}

int partial_stride(const Ctx &c) { return stage_nsb(c, kFormLds); }

// 4-D tiles of the LDS form's 64-site blocks, when 64 sites are whole y rows and
// the tile divides the lattice: 4 z-planes x 4 timeslices (8 x 8 for FP64).
// Measured on 32^3 x 64 at 128 RHS with the items in dispatch order, per stage
// pair: FP16N 15.59 ms (memory order 15.76, 2 x 2 15.96, 8 x 8 15.60), FP64 53.7
// ms (2 x 2 55.8, 4 x 4 54.6, memory order 55.9).
static void lds_block_tiles(const Ctx &c, const StageSpec &s, StageArgs &a) {
    a.nyb = a.tz = a.tt = 0;
    const int rows = kLdsSites % c.g.lxh == 0 ? kLdsSites / c.g.lxh : 0;
    if (s.form != kFormLds || rows == 0 || c.g.ly % rows != 0) return;
    for (int t : {s.prec == LAPH_F64 ? 8 : 4, 4, 2}) {
        if (c.g.lz % t == 0 && c.g.lt % t == 0) {
            a.nyb = c.g.ly / rows;
            a.tz = a.tt = t;
            return;
        }
    }
}

laph_status launch_stage(const Ctx &c, const StageSpec &s) {
    StageArgs a;
    a.g = c.g;
    a.gp = c.gp;
    a.out_parity = s.out_parity;
    a.in = s.in;
    a.out = s.out;
    a.y = s.y;
    a.y2 = s.y2;
    a.z = s.z;
    a.w = s.w;
    a.a = s.a;
    a.a2 = s.a2;
    a.b = s.b;
    a.c = s.c;
    a.clover = s.clover ? c.clover_inv(s.prec, 0, s.out_parity) : nullptr;
    a.clover_mass_stride = c.clover_inv_mass_stride(s.prec);
    a.tile_slots = s.tiles.slots;
    a.tile_mass = s.tiles.mass;
    a.ntiles = s.tiles.ntiles;
    a.ntiles_max = s.tiles.ntiles_max;
    a.nsb = stage_nsb(c, s.form);
    a.pstride = s.pstride;
    a.site_major = s.site_major;
    a.grid_cap = s.grid_cap;
    lds_block_tiles(c, s, a);
    a.dispatch_order = s.form == kFormLds ? 1 : 0;
    a.win = s.win;
    a.clover_term = (s.red == 4 || s.red == 5) ? c.clover_term(s.out_parity) : nullptr;
    a.diag = c.mass_diag();
    a.flag_filter = s.flagged;
    a.one = 1.0f;
    a.st = s.slots;
    a.partials = s.partials;
    if (a.ntiles_max <= 0) return LAPH_OK;
    if (s.red && s.pstride < a.nsb) return set_error(LAPH_ERR_INVALID, "partial-sum stride too small");
    // a skipped site block would leave its partial sums unwritten
    if (s.red && s.win.n > 0) return set_error(LAPH_ERR_INVALID, "site window on a reducing stage");
    bool ok = false;
    if (s.form == kFormLds) {
        if (s.prec == LAPH_F64)
            ok = launch_stage_lds_f64(s, a, c.stream);
        else if (s.prec == LAPH_F32)
            ok = launch_stage_lds_f32(s, a, c.stream);
        else if (s.prec == LAPH_F16N)
            ok = launch_stage_lds_f16(s, a, c.stream);
    } else if (s.prec == LAPH_F64) {
        ok = launch_stage_f64(s, a, c.stream);
    } else if (s.prec == LAPH_F32) {
        ok = launch_stage_f32(s, a, c.stream);
    } else if (s.prec == LAPH_F16N) {
        ok = launch_stage_f16(s, a, c.stream);
    }
    if (!ok) return set_error(LAPH_ERR_INVALID, "unsupported stencil stage combination");
    return check_launch("stage_kernel");
}

// ---------------------------------------------------------------------------
// clover apply: out = a*y + b * M in, M = A or A^-1 of one parity
// ---------------------------------------------------------------------------
struct CloverArgs {
    int vh;
    Operand in, out, y;
    double a, b;
    const char *mat;           // inverse: FP64/FP32 inverse of mass 0; else the FP64 clover term
    size_t mass_stride;
    int inverse;
    const double *diag;        // per mass: 4 + m0 (used when !inverse)
    const int *slot_list;
    const int *slot_mass;
    int mass_idx;
    int n;
    SiteWindow win;            // sites computed (the others untouched)
};

// One thread per site; a block row takes kCloverRhs RHS in turn, so the clover
// blocks of its sites come from HBM once and from the caches for the other RHS
// (a grid row per RHS streamed the whole clover field once per RHS).
constexpr int kCloverRhs = 4;

template <class P, bool POST>
__global__ __launch_bounds__(kBlock) void clover_kernel(CloverArgs A) {
    using R = typename P::real;
    const int h = blockIdx.x * kBlock + threadIdx.x;
    if (h >= A.vh || !in_window(A.win, h, A.vh)) return;
#pragma unroll 1
    for (int jj = 0; jj < kCloverRhs; ++jj) {
        const int j = blockIdx.y * kCloverRhs + jj;
        if (j >= A.n) break;
        const int slot = A.slot_list ? A.slot_list[j] : j;
        const int mass = A.slot_mass ? A.slot_mass[slot] : A.mass_idx;
        cplx<R> in[12], out[12];
        SpinorIO<P>::load(A.in.at(slot), A.vh, h, in);
#pragma unroll
        for (int blk = 0; blk < 2; ++blk) {
            R mm[36];
            if (A.inverse) {
                CloverIO<P>::load(A.mat + (size_t)mass * A.mass_stride, blk, A.vh, h, mm);
                herm6_apply(mm, &in[6 * blk], &out[6 * blk]);
            } else {
                // the clover term is kept in FP64 only; A = (4 + m0) + term
                double md[36];
                CloverIO<F64>::load(A.mat, blk, A.vh, h, md);
#pragma unroll
                for (int k = 0; k < 36; ++k) mm[k] = R(md[k]);
                herm6_apply(mm, &in[6 * blk], &out[6 * blk], R(A.diag[mass]));
            }
        }
        const R bb = R(A.b);
#pragma unroll
        for (int c = 0; c < 12; ++c) out[c] = bb * out[c];
        if (POST) {
            cplx<R> yy[12];
            SpinorIO<P>::load(A.y.at(slot), A.vh, h, yy);
            const R aa = R(A.a);
#pragma unroll
            for (int c = 0; c < 12; ++c) out[c] = out[c] + aa * yy[c];
        }
        SpinorIO<P>::store(A.out.at(slot), A.vh, h, out);
    }
}

laph_status launch_clover(const Ctx &c, const CloverSpec &s) {
    if (s.n <= 0) return LAPH_OK;
    CloverArgs a;
    a.vh = c.g.vh;
    a.in = s.in;
    a.out = s.out;
    a.y = s.y;
    a.a = s.a;
    a.b = s.b;
    a.inverse = s.inverse;
    a.mat = s.inverse ? c.clover_inv(s.prec, 0, s.parity) : c.clover_term(s.parity);
    a.mass_stride = c.clover_inv_mass_stride(s.prec);
    a.diag = c.mass_diag();
    a.slot_list = s.slot_list;
    a.slot_mass = s.slot_mass;
    a.mass_idx = s.mass_idx;
    a.n = s.n;
    a.win = s.win;
    dim3 grid((c.g.vh + kBlock - 1) / kBlock, (s.n + kCloverRhs - 1) / kCloverRhs);
#define LAPH_CL(PT)                                                                                   \
    if (s.post)                                                                                       \
        hipLaunchKernelGGL((clover_kernel<PT, true>), grid, dim3(kBlock), 0, c.stream, a);           \
    else                                                                                              \
        hipLaunchKernelGGL((clover_kernel<PT, false>), grid, dim3(kBlock), 0, c.stream, a);
    if (s.prec == LAPH_F64) {
        LAPH_CL(F64)
    } else if (s.prec == LAPH_F32) {
        LAPH_CL(F32)
    } else {
        LAPH_CL(F16N)
    }
#undef LAPH_CL
    return check_launch("clover_kernel");
}

}  // namespace laph
