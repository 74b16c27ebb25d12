// Declarations of the solver's vector kernels (blas.hip).
#pragma once

#include "laph_host.h"

namespace laph {

enum { kModeAll = 0, kModeActive = 1, kModeFlagged = 2 };
enum { kFinAlpha, kFinOmega, kFinRho, kFinUpdate, kFinRho2, kFinInit, kFinBnorm, kFinR64, kFinTrueRes };

struct BlasArgs {
    int vh = 0;
    int nsb = 0;                 // site blocks of 256 (partials written per quantity per slot)
    int pstride = 0;             // partial-sum stride per quantity per slot
    const int *list = nullptr;   // slot list
    const int *nlist = nullptr;  // device scalar: entries in use
    int nlist_max = 0;           // grid size
    SlotState *st = nullptr;
    double *partials = nullptr;  // [slot][3][pstride]
    Operand r, rh, p, v, t, x;   // inner-precision vectors (x: the x_lo precision)
    Operand x64, r64;            // FP64 solution and residual
    const int *flist = nullptr;  // flagged mode: slots taking a reliable update
    const int *nflist = nullptr; // device scalar: entries of flist
    SiteWindow win;              // norm2 / copy64: the sources are zero outside it (not read)
};

// Input / output of the flagged-slot compaction (blas_flag_tiles).
struct FlagArgs {
    const int *tile_slots = nullptr;   // static FP64 tiles [ntiles][nr], grouped by mass
    const int *tile_mass = nullptr;
    const int *ntiles = nullptr;       // device scalar
    int nr = 1;
    const SlotState *st = nullptr;
    int *out_slots = nullptr, *out_mass = nullptr, *out_ntiles = nullptr;   // flagged tiles
    int *flist = nullptr, *nflist = nullptr;                                // flagged slots
};

struct FinArgs {
    const int *list = nullptr;
    const int *nlist = nullptr;
    int nlist_max = 0;
    int nsb = 0;        // partials to sum (the producing kernel's site blocks)
    int pstride = 0;    // partial-sum stride per quantity per slot
    SlotState *st = nullptr;
    const double *partials = nullptr;
    int max_restarts = 10;
};

laph_status blas_p_update(const Ctx &c, const BlasArgs &a, int prec);
laph_status blas_s_update(const Ctx &c, const BlasArgs &a, int prec);
laph_status blas_xr_update(const Ctx &c, const BlasArgs &a, int prec);
laph_status blas_accumulate(const Ctx &c, const BlasArgs &a, int prec, int mode);
laph_status blas_lower(const Ctx &c, const BlasArgs &a, int prec, int mode, int init);
laph_status blas_norm2(const Ctx &c, const BlasArgs &a, Operand v1, Operand v2, int mode);
laph_status blas_copy64(const Ctx &c, const BlasArgs &a, Operand dst, Operand src, int mode);
laph_status blas_flag_tiles(const Ctx &c, const FlagArgs &f);
laph_status blas_finalize(const Ctx &c, const FinArgs &f, int what);

}  // namespace laph
