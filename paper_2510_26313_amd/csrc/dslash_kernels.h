// Even-odd Wilson-clover stencil stages for gfx950.
//
// One thread owns one output site of the output parity and NR right-hand sides
// (a "tile" of RHS that share one mass).  For each of the 8 hops the link is
// loaded once and applied to the NR neighbour spinors, so the link and clover
// traffic is amortised over the tile.  The (1 -/+ gamma_mu) projection halves
// the colour work: only two colour vectors are multiplied by the link and the
// other two spin rows are rebuilt from them.  The clover inverse of the output
// site, the xpay terms and the solver's inner products are fused into the
// epilogue, with FP64 per-block partial sums (wave shuffles, then LDS).
//
// Workgroup -> (site block, tile) uses an XCD-aware remap: workgroups that one
// XCD receives are consecutive logical ids, and the tile index runs fastest,
// so all tiles of a site block run on one XCD and share its L2 for the links.
#pragma once

#include <type_traits>

#include "laph_host.h"

namespace laph {

constexpr int kBlock = 256;

// Register budget of the stencil kernels: ask for at least this many waves per
// SIMD so the compiler keeps the kernel under 512 / N VGPRs (memory latency is
// hidden by occupancy; the accumulators of a 4-RHS tile still fit).
#ifndef LAPH_STAGE_WAVES
#define LAPH_STAGE_WAVES 1
#endif
#define LAPH_STAGE_OCCUPANCY __attribute__((amdgpu_waves_per_eu(LAPH_STAGE_WAVES)))

struct StageArgs {
    Geom g;
    GaugePtrs gp;
    int out_parity;
    Operand in, out, y, y2, z, w;
    double a, a2, b, c;
    const char *clover;
    size_t clover_mass_stride;
    const int *tile_slots;
    const int *tile_mass;
    const int *ntiles;
    int ntiles_max;
    int nsb;
    int pstride;
    int site_major;
    const SlotState *st;
    double *partials;
    float one;   // 1.0f, opaque to the compiler (keeps FP16N projections as mixed-precision FMAs)
    int grid_cap;   // launch only: at most this many workgroups (0: one per item)
    int flag_filter;   // LDS form: skip slots not flagged for a reliable update
    // LDS form: order of the 64-site blocks as 4-D tiles (nyb blocks of y rows x
    // tz z-planes x tt timeslices); tz == 0: memory order
    int nyb, tz, tt;
    int dispatch_order;   // 1: items in dispatch order (see stage_item_range); 0: per-XCD ranges
    SiteWindow win;       // output sites computed; the others are neither read nor written
    // reductions 4 and 5 (FP64 LDS form): the clover term of the output parity and the
    // per-mass diagonal 4 + m0 (|v - A out|^2; a y + b H in - A y2)
    const char *clover_term;
    const double *diag;
};

// Work items of a stage launch are (site block, tile) pairs of the live tiles:
// W = ntiles * nsb with ntiles read on the device.  Workgroups are dispatched
// round-robin over the 8 XCDs (workgroup b runs on XCD b % 8).  Per-XCD ranges
// (the register form): the items are split into 8 contiguous ranges, one per XCD,
// and the workgroups of an XCD walk its range with a stride of gridDim.x / 8, so an
// XCD's L2 holds the neighbour rows of its own blocks.  Dispatch order (the LDS
// form): workgroup b takes items b, b + gridDim.x, ..., so all XCDs work on the same
// stretch of the lattice at once and share its neighbour rows and links through the
// Infinity Cache.  Measured at 32^3 x 64, stage pairs at 128 RHS: FP16N 15.59 against
// 15.84 ms, FP32 26.3 against 30.5 ms, FP64 53.7 against 59.0 ms (with 8 x 8 block
// tiles); 4 and 8 RHS -4 to -6 %; the register form at 1-16 RHS is up to a third slower
// in dispatch order.  A grid of W_max workgroups takes at most one item each; a
// smaller grid (launches whose live tile count is known only on the device) loops, so
// no workgroup of a retired or unflagged tile is scheduled.  Site-major: each tile
// sweeps all site blocks (neighbouring site blocks, whose spinors are each other's
// hop inputs, run close in time); tile-major: the tiles of one site block are
// consecutive (they share its links in the caches).
__device__ __forceinline__ void stage_item_range(int W, int dispatch_order, int &first, int &end, int &step) {
    if (dispatch_order) {
        first = blockIdx.x;
        end = W;
        step = gridDim.x;
        return;
    }
    const int per = gridDim.x >> 3;   // launches pad the grid to a multiple of 8
    const int xcd = blockIdx.x & 7, k = blockIdx.x >> 3;
    const int chunk = (W + 7) >> 3;
    first = xcd * chunk + k;
    end = min(W, (xcd + 1) * chunk);
    step = per;
}
__device__ __forceinline__ void stage_item(int w, int site_major, int nsb, int ntiles, int &sb, int &tile) {
    if (site_major) {
        tile = w / nsb;
        sb = w - tile * nsb;
    } else {
        sb = w / ntiles;
        tile = w - sb * ntiles;
    }
}
// Physical site block of the L-th block in the tiled order: within a tile the y
// blocks run fastest, then tz z-planes, then tt timeslices; tiles go in z, then t.
// Blocks that run at the same time then hold each other's z and t neighbours,
// which stay in L2 instead of being fetched again from HBM.
__device__ __forceinline__ int tiled_block(int L, int nyb, int tz, int tt, int lz) {
    if (tz == 0) return L;
    const int yb = L % nyb;
    int r = L / nyb;
    const int zl = r % tz;
    r /= tz;
    const int tl = r % tt;
    r /= tt;
    const int nzt = lz / tz;
    const int ztile = r % nzt;
    const int ttile = r / nzt;
    return ((ttile * tt + tl) * lz + ztile * tz + zl) * nyb + yb;
}
// grid of a stage launch: every item, or at most cap workgroups (cap > 0)
inline int stage_grid(int items_max, int cap) {
    int n = cap > 0 && cap < items_max ? cap : items_max;
    return pad8(n > 0 ? n : 1);
}

// --- spin projection: (1 + S gamma_mu) psi = (h0, h1, row2(h), row3(h)) --------
// gamma_x rows: (i p3, i p2, -i p1, -i p0); gamma_y: (-p3, p2, p1, -p0);
// gamma_z: (i p2, -i p3, -i p0, i p1); gamma_t: (p2, p3, p0, p1).
template <int S, class R>
__device__ __forceinline__ cplx<R> s_i(cplx<R> z) {  // S * i * z
    return S > 0 ? mul_i(z) : mul_mi(z);
}
template <int S, class R>
__device__ __forceinline__ cplx<R> s_1(cplx<R> z) {  // S * z
    return S > 0 ? z : cplx<R>{-z.re, -z.im};
}

template <int MU, int S, class R>
__device__ __forceinline__ void spin_project(const cplx<R> (&p)[12], cplx<R> (&h)[6]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (MU == 0) {
            h[a] = p[a] + s_i<S>(p[9 + a]);
            h[3 + a] = p[3 + a] + s_i<S>(p[6 + a]);
        } else if (MU == 1) {
            h[a] = p[a] - s_1<S>(p[9 + a]);
            h[3 + a] = p[3 + a] + s_1<S>(p[6 + a]);
        } else if (MU == 2) {
            h[a] = p[a] + s_i<S>(p[6 + a]);
            h[3 + a] = p[3 + a] - s_i<S>(p[9 + a]);
        } else {
            h[a] = p[a] + s_1<S>(p[6 + a]);
            h[3 + a] = p[3 + a] + s_1<S>(p[9 + a]);
        }
    }
}

// The same projection for an FP16N neighbour, computed from its binary16 codes:
// x + c y with c in {1, -1, i, -i} per real part as one mixed-precision fused
// multiply-add (binary16 inputs, binary32 result; exact inputs, one rounding --
// the value of converting both and adding).  `one` is 1.0f.
template <int C>
__device__ __forceinline__ cplx<float> proj_mix(_Float16 xr, _Float16 xi, _Float16 yr, _Float16 yi, float one) {
    if (C == 1) return {fmaf((float)yr, one, (float)xr), fmaf((float)yi, one, (float)xi)};
    if (C == -1) return {fmaf((float)yr, -one, (float)xr), fmaf((float)yi, -one, (float)xi)};
    if (C == 2) return {fmaf((float)yi, -one, (float)xr), fmaf((float)yr, one, (float)xi)};   // + i y
    return {fmaf((float)yi, one, (float)xr), fmaf((float)yr, -one, (float)xi)};               // - i y
}

template <int MU, int S>
__device__ __forceinline__ void spin_project_codes(const half8 (&q)[3], float one, cplx<float> (&h)[6]) {
    // component c (= 3 spin + colour) has its real part at q[c / 4][2 (c % 4)]
#define LAPH_Q(c) q[(c) >> 2][2 * ((c)&3)], q[(c) >> 2][2 * ((c)&3) + 1]
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (MU == 0) {
            h[a] = proj_mix<2 * S>(LAPH_Q(a), LAPH_Q(9 + a), one);
            h[3 + a] = proj_mix<2 * S>(LAPH_Q(3 + a), LAPH_Q(6 + a), one);
        } else if (MU == 1) {
            h[a] = proj_mix<-S>(LAPH_Q(a), LAPH_Q(9 + a), one);
            h[3 + a] = proj_mix<S>(LAPH_Q(3 + a), LAPH_Q(6 + a), one);
        } else if (MU == 2) {
            h[a] = proj_mix<2 * S>(LAPH_Q(a), LAPH_Q(6 + a), one);
            h[3 + a] = proj_mix<-2 * S>(LAPH_Q(3 + a), LAPH_Q(9 + a), one);
        } else {
            h[a] = proj_mix<S>(LAPH_Q(a), LAPH_Q(6 + a), one);
            h[3 + a] = proj_mix<S>(LAPH_Q(3 + a), LAPH_Q(9 + a), one);
        }
    }
#undef LAPH_Q
}

// Load and project a neighbour half-spinor; returns the factor still to apply
// (the FP16N site norm, 1 otherwise).
template <class P, int MU, int S>
__device__ __forceinline__ typename P::real load_project(const char *hv, int vh, int h, float one,
                                                         cplx<typename P::real> (&hs)[6]) {
    using R = typename P::real;
    if constexpr (SpinorIO<P>::kNorm) {
        half8 q[3];
        float n;
        SpinorIO<P>::load_codes(hv, vh, h, q, n);
        spin_project_codes<MU, S>(q, one, hs);
        return n;
    } else {
        cplx<R> psi[12];
        R n;
        SpinorIO<P>::load_unscaled(hv, vh, h, psi, n);
        spin_project<MU, S>(psi, hs);
        return R(1);
    }
}

// An FP32 half-vector into FP64 arithmetic: the values are widened before the spin
// projection, so the FP64 stage is exact to FP64 rounding in its FP32 inputs.
template <int MU, int S>
__device__ __forceinline__ double load_project_widened(const char *hv, int vh, int h, cplx<double> (&hs)[6]) {
    cplx<float> pf[12];
    SpinorIO<F32>::load(hv, vh, h, pf);
    cplx<double> psi[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) psi[c] = {double(pf[c].re), double(pf[c].im)};
    spin_project<MU, S>(psi, hs);
    return 1.0;
}

// acc += sc * (u, row2(u), row3(u)): the lower spin components of (1 + S gamma_mu)
// follow from the upper ones; the scale sc (FP16 site norm, time-boundary sign)
// is folded into the fused multiply-adds.
template <int MU, int S, class R>
__device__ __forceinline__ void spin_accumulate(cplx<R> (&acc)[12], const cplx<R> (&u)[6], R sc) {
    // S * i * z scaled: (-S sc z.im, S sc z.re); S * z scaled: (S sc z.re, S sc z.im)
    const R ss = S > 0 ? sc : -sc;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        acc[a] = caxpy(sc, u[a], acc[a]);
        acc[3 + a] = caxpy(sc, u[3 + a], acc[3 + a]);
        if (MU == 0) {   // lower = -S i (u1, u0)
            acc[6 + a] = {ffma(ss, u[3 + a].im, acc[6 + a].re), ffma(-ss, u[3 + a].re, acc[6 + a].im)};
            acc[9 + a] = {ffma(ss, u[a].im, acc[9 + a].re), ffma(-ss, u[a].re, acc[9 + a].im)};
        } else if (MU == 1) {   // lower = (S u1, -S u0)
            acc[6 + a] = caxpy(ss, u[3 + a], acc[6 + a]);
            acc[9 + a] = caxpy(-ss, u[a], acc[9 + a]);
        } else if (MU == 2) {   // lower = (-S i u0, S i u1)
            acc[6 + a] = {ffma(ss, u[a].im, acc[6 + a].re), ffma(-ss, u[a].re, acc[6 + a].im)};
            acc[9 + a] = {ffma(-ss, u[3 + a].im, acc[9 + a].re), ffma(ss, u[3 + a].re, acc[9 + a].im)};
        } else {   // lower = (S u0, S u1)
            acc[6 + a] = caxpy(ss, u[a], acc[6 + a]);
            acc[9 + a] = caxpy(ss, u[3 + a], acc[9 + a]);
        }
    }
}

// u = L h  (ADJ: L^dagger h) for both colour vectors of the half spinor; CHAIN:
// fused multiply-add chains (cfma) instead of sums of products (cmac)
template <bool ADJ, class R, bool CHAIN = false>
__device__ __forceinline__ void colour_mul(const cplx<R> (&L)[9], const cplx<R> (&h)[6], cplx<R> (&u)[6]) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cplx<R> s = ADJ ? cmul1_conj(L[a], h[3 * j]) : cmul1(L[a * 3], h[3 * j]);
#pragma unroll
            for (int b = 1; b < 3; ++b) {
                if (ADJ) {
                    if (CHAIN)
                        cfma_conj(s, L[b * 3 + a], h[3 * j + b]);
                    else
                        cmac_conj(s, L[b * 3 + a], h[3 * j + b]);
                } else {
                    if (CHAIN)
                        cfma(s, L[a * 3 + b], h[3 * j + b]);
                    else
                        cmac(s, L[a * 3 + b], h[3 * j + b]);
                }
            }
            u[3 * j + a] = s;
        }
    }
}

// One hop (forward: FWD, link U_mu(x), neighbour x + mu; backward: link
// U_mu(x - mu)^dagger, neighbour x - mu) for the NR right-hand sides of the tile.
// The spin projection is linear, so an FP16N neighbour is projected from its
// codes and its norm is applied together with the boundary sign after the
// colour product (12 multiplies instead of 24).
template <class P, int NR, int MU, bool DAG, bool FWD>
__device__ __forceinline__ void hop_dir(const StageArgs &A, int p, int h, const int (&x)[4],
                                        const int (&slots)[NR], cplx<typename P::real> (&acc)[NR][12]) {
    using R = typename P::real;
    constexpr int S = (FWD != DAG) ? -1 : 1;     // (1 + S gamma_mu)
    const Geom &g = A.g;
    const int ext = MU == 0 ? g.lx : (MU == 1 ? g.ly : (MU == 2 ? g.lz : g.lt));
    int n[4] = {x[0], x[1], x[2], x[3]};
    bool wrap = false;
    if (FWD) {
        n[MU] = x[MU] + 1;
        if (n[MU] == ext) { n[MU] = 0; wrap = true; }
    } else {
        n[MU] = x[MU] - 1;
        if (n[MU] < 0) { n[MU] = ext - 1; wrap = true; }
    }
    const R eta = (MU == 3 && wrap && g.antiperiodic) ? R(-1) : R(1);
    const int hn = cb_index(g, n[0], n[1], n[2], n[3]);
    cplx<R> L[9];
    if (FWD)
        GaugeIO<P>::load(A.gp, p, MU, g.vh, h, L);
    else
        GaugeIO<P>::load(A.gp, 1 - p, MU, g.vh, hn, L);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (slots[r] < 0) continue;
        cplx<R> hs[6], u[6];
        const R nrm = load_project<P, MU, S>(A.in.at(slots[r]), g.vh, hn, A.one, hs);
        colour_mul<!FWD>(L, hs, u);
        spin_accumulate<MU, S>(acc[r], u, SpinorIO<P>::kNorm ? eta * nrm : eta);
    }
}

// Keep the instruction scheduler from hoisting the loads of all eight hops to
// the top of the kernel: that schedule needs several hundred VGPRs (occupancy 1
// or spills); latency is hidden across waves instead.
__device__ __forceinline__ void hop_fence() { __builtin_amdgcn_sched_barrier(0); }

template <class P, int NR, int MU, bool DAG>
__device__ __forceinline__ void hop_mu(const StageArgs &A, int p, int h, const int (&x)[4],
                                       const int (&slots)[NR], cplx<typename P::real> (&acc)[NR][12]) {
    hop_dir<P, NR, MU, DAG, true>(A, p, h, x, slots, acc);
    hop_fence();
    hop_dir<P, NR, MU, DAG, false>(A, p, h, x, slots, acc);
    hop_fence();
}

// FP64 block reduction of NV values per thread; thread 0 writes NV partials.
template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&v)[NV], double *dst, size_t q_stride) {
    __shared__ double red[kBlock / 64][NV > 0 ? NV : 1];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = v[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        v[q] = s;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) red[wave][q] = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double s = 0;
            for (int wv = 0; wv < kBlock / 64; ++wv) s += red[wv][q];
            dst[q * q_stride] = s;
        }
    }
}

// One work item: NR right-hand sides of a tile on kBlock sites.
template <class P, int NR, bool DAG, bool CLOVER, bool PRE, int POST, int RED, bool FLAGGED>
__device__ __forceinline__ void stage_body(const StageArgs &A, int sb, int tile) {
    using R = typename P::real;
    int slots[NR];
    bool any = false;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        int s = A.tile_slots[tile * NR + r];
        if (FLAGGED && s >= 0 && !(A.st[s].flag != 0 && A.st[s].status == LAPH_RHS_ACTIVE)) s = -1;
        slots[r] = s;
        any |= s >= 0;
    }
    if (!any) return;
    const Geom &g = A.g;
    if (block_outside(A.win, sb * kBlock, min(kBlock, g.vh - sb * kBlock), g.vh)) return;   // uniform
    const int p = A.out_parity;
    const int h = sb * kBlock + threadIdx.x;
    const bool valid = h < g.vh && in_window(A.win, h, g.vh);
    constexpr int NQ = RED == 1 ? 2 : (RED == 2 ? 3 : (RED == 3 ? 1 : 0));
    double part[NR][NQ > 0 ? NQ : 1];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int q = 0; q < (NQ > 0 ? NQ : 1); ++q) part[r][q] = 0.0;

    if (valid) {
        int x[4];
        site_coords(g, p, h, x[0], x[1], x[2], x[3]);
        cplx<R> acc[NR][12];
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int c = 0; c < 12; ++c) acc[r][c] = {R(0), R(0)};
        hop_mu<P, NR, 0, DAG>(A, p, h, x, slots, acc);
        hop_mu<P, NR, 1, DAG>(A, p, h, x, slots, acc);
        hop_mu<P, NR, 2, DAG>(A, p, h, x, slots, acc);
        hop_mu<P, NR, 3, DAG>(A, p, h, x, slots, acc);

        if (PRE) {
            const R cz = R(A.c);
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                if (slots[r] < 0) continue;
                cplx<R> zz[12];
                SpinorIO<P>::load(A.z.at(slots[r]), g.vh, h, zz);
#pragma unroll
                for (int c = 0; c < 12; ++c) acc[r][c] = acc[r][c] + cz * zz[c];
            }
        }
        if (CLOVER) {
            const char *cl = A.clover + (size_t)A.tile_mass[tile] * A.clover_mass_stride;
#pragma unroll
            for (int blk = 0; blk < 2; ++blk) {
                R m[36];
                CloverIO<P>::load(cl, blk, g.vh, h, m);
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    cplx<R> o[6];
                    herm6_apply(m, &acc[r][6 * blk], o);
#pragma unroll
                    for (int i = 0; i < 6; ++i) acc[r][6 * blk + i] = o[i];
                }
            }
        }
        const R bb = R(A.b), aa = R(A.a), aa2 = R(A.a2);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (slots[r] < 0) continue;
            cplx<R> res[12], yy[12];
#pragma unroll
            for (int c = 0; c < 12; ++c) res[c] = bb * acc[r][c];
            if (POST >= 1) {
                SpinorIO<P>::load(A.y.at(slots[r]), g.vh, h, yy);
#pragma unroll
                for (int c = 0; c < 12; ++c) res[c] = res[c] + aa * yy[c];
            }
            if (POST >= 2) {
                cplx<R> y2[12];
                SpinorIO<P>::load(A.y2.at(slots[r]), g.vh, h, y2);
#pragma unroll
                for (int c = 0; c < 12; ++c) res[c] = res[c] + aa2 * y2[c];
            }
            SpinorIO<P>::store(A.out.at(slots[r]), g.vh, h, res);
            if (RED == 1) {
                cplx<R> ww[12];
                SpinorIO<P>::load(A.w.at(slots[r]), g.vh, h, ww);
                cplx<R> d = {R(0), R(0)};
#pragma unroll
                for (int c = 0; c < 12; ++c) cmac_conj(d, ww[c], res[c]);
                part[r][0] = (double)d.re;
                part[r][1] = (double)d.im;
            } else if (RED == 2) {
                cplx<R> d = {R(0), R(0)};
                R n2 = R(0);
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    cmac_conj(d, res[c], yy[c]);
                    n2 += res[c].re * res[c].re + res[c].im * res[c].im;
                }
                part[r][0] = (double)d.re;
                part[r][1] = (double)d.im;
                part[r][2] = (double)n2;
            } else if (RED == 3) {
                R n2 = R(0);
#pragma unroll
                for (int c = 0; c < 12; ++c) n2 += res[c].re * res[c].re + res[c].im * res[c].im;
                part[r][0] = (double)n2;
            }
        }
    }
    if constexpr (NQ > 0) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            double v[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) v[q] = part[r][q];
            // every thread of the block takes part in the reduction (uniform branch)
            if (slots[r] >= 0) {
                block_reduce_store<NQ>(v, A.partials + ((size_t)slots[r] * 3) * A.pstride + sb, (size_t)A.pstride);
                __syncthreads();
            }
        }
    }
}

template <class P, int NR, bool DAG, bool CLOVER, bool PRE, int POST, int RED, bool FLAGGED>
__global__ __launch_bounds__(kBlock) LAPH_STAGE_OCCUPANCY void stage_kernel(StageArgs A) {
    const int nt = *A.ntiles;
    int first, end, step;
    stage_item_range(nt * A.nsb, A.dispatch_order, first, end, step);
    for (int w = first; w < end; w += step) {
        int sb, tile;
        stage_item(w, A.site_major, A.nsb, nt, sb, tile);
        stage_body<P, NR, DAG, CLOVER, PRE, POST, RED, FLAGGED>(A, sb, tile);
    }
}


// ---------------------------------------------------------------------------
// dispatch (instantiated per precision in dslash_f64/f32/f16.hip)
// ---------------------------------------------------------------------------
template <class P, int NR, bool DAG, bool CLOVER, bool PRE, int POST, int RED, bool FL>
inline void launch_t(const StageArgs &a, hipStream_t st) {
    const int nblk = stage_grid(a.nsb * a.ntiles_max, a.grid_cap);
    hipLaunchKernelGGL((stage_kernel<P, NR, DAG, CLOVER, PRE, POST, RED, FL>), dim3(nblk), dim3(kBlock), 0, st, a);
}

// The (clover, pre, post, red) combinations the library uses.
template <class P, int NR, bool DAG, bool FL>
inline bool launch_combo(const StageSpec &s, const StageArgs &a, hipStream_t st) {
    constexpr bool is64 = std::is_same<P, F64>::value;
    const int key = s.clover * 1000 + s.pre * 100 + s.post * 10 + s.red;
    if constexpr (FL) {
        // masked reliable-update stages exist in FP64 only
        if constexpr (is64) {
            if (key == 1000) { launch_t<P, NR, DAG, true, false, 0, 0, FL>(a, st); return true; }
            if (key == 1023) { launch_t<P, NR, DAG, true, false, 2, 3, FL>(a, st); return true; }
        }
        return false;
    } else {
        switch (key) {
            case 1000: launch_t<P, NR, DAG, true, false, 0, 0, FL>(a, st); return true;     // A^-1 H in
            case 1011: launch_t<P, NR, DAG, true, false, 1, 1, FL>(a, st); return true;     // v = p - A^-1 H t, <r^, v>
            case 1012: launch_t<P, NR, DAG, true, false, 1, 2, FL>(a, st); return true;     // t = s - A^-1 H t, <t,s>,|t|^2
            default: break;
        }
        if constexpr (NR == 1) {
            if (key == 0) { launch_t<P, NR, DAG, false, false, 0, 0, FL>(a, st); return true; }  // bare hop
        }
        if constexpr (is64) {
            switch (key) {
                case 0: launch_t<P, NR, DAG, false, false, 0, 0, FL>(a, st); return true;
                case 10: launch_t<P, NR, DAG, false, false, 1, 0, FL>(a, st); return true;    // y + b H in
                case 13: launch_t<P, NR, DAG, false, false, 1, 3, FL>(a, st); return true;    // residual part
                case 1023: launch_t<P, NR, DAG, true, false, 2, 3, FL>(a, st); return true;   // r64, |r64|^2
                case 1100: launch_t<P, NR, DAG, true, true, 0, 0, FL>(a, st); return true;    // A^-1 (c z + H in)
                default: break;
            }
        }
        return false;
    }
}

template <class P, int NR>
inline bool launch_nr(const StageSpec &s, const StageArgs &a, hipStream_t st) {
    if (s.dagger)
        return s.flagged ? launch_combo<P, NR, true, true>(s, a, st) : launch_combo<P, NR, true, false>(s, a, st);
    return s.flagged ? launch_combo<P, NR, false, true>(s, a, st) : launch_combo<P, NR, false, false>(s, a, st);
}

template <class P>
inline bool launch_p(const StageSpec &s, const StageArgs &a, hipStream_t st) {
    switch (s.tiles.nr) {
        case 1: return launch_nr<P, 1>(s, a, st);
        case 2: return launch_nr<P, 2>(s, a, st);
        case 4: return launch_nr<P, 4>(s, a, st);
        default: return false;
    }
}


bool launch_stage_f64(const StageSpec &s, const StageArgs &a, hipStream_t st);
bool launch_stage_f32(const StageSpec &s, const StageArgs &a, hipStream_t st);
bool launch_stage_f16(const StageSpec &s, const StageArgs &a, hipStream_t st);

}  // namespace laph
