// Even-odd stencil stage, RHS-parallel form with the links staged in LDS.
//
// A workgroup owns 64 output sites and a tile of 4*RW right-hand sides of one
// mass.  Phase 1: its four waves compute the 8 neighbour indices of the 64
// sites and load, decompress (third row) and store the 8 links per site in
// LDS, already transposed for the backward hops and multiplied by the
// time-boundary sign.  Phase 2: each wave takes one RHS at a time (RW rounds);
// a lane owns one site, so its accumulator is a single 12-component spinor,
// the neighbour spinor loads of a wave are coalesced (consecutive sites), and
// every link staged in LDS is reused by all 4*RW RHS of the tile.  Compared
// with the register-tile form this keeps the VGPR count low (high occupancy
// hides the neighbour-gather latency) while still reading each link once per
// tile.  Inner products are reduced per wave (one partial per 64 sites).
#pragma once

#include "dslash_kernels.h"

namespace laph {

constexpr int kLdsSites = 64;

// One hop for one RHS: neighbour index and link (already L or L^dagger, times the
// boundary sign) come from LDS; an FP16N neighbour is projected from its codes
// and scaled by its norm after the colour product.  WIDEN: an FP32 input half-vector
// in an FP64 stage.
template <class P, int MU, bool DAG, bool FWD, bool WIDEN = false>
__device__ __forceinline__ void lds_hop(const char *src, int vh, const typename P::real (&lnk)[8][18][kLdsSites],
                                        const int (&nbr)[8][kLdsSites], int lane, float one,
                                        cplx<typename P::real> (&acc)[12]) {
    using R = typename P::real;
    constexpr int hop = 2 * MU + (FWD ? 0 : 1);
    constexpr int S = (FWD != DAG) ? -1 : 1;
    const int hn = nbr[hop][lane];
    cplx<R> hs[6], u[6], L[9];
    R nrm;
    if constexpr (WIDEN)
        nrm = load_project_widened<MU, S>(src, vh, hn, hs);
    else
        nrm = load_project<P, MU, S>(src, vh, hn, one, hs);
#pragma unroll
    for (int k = 0; k < 9; ++k) L[k] = {lnk[hop][2 * k][lane], lnk[hop][2 * k + 1][lane]};
    colour_mul<false, R, (sizeof(R) == 4)>(L, hs, u);
    spin_accumulate<MU, S>(acc, u, nrm);
}

// Barrier between the phases of one RHS (after each hop direction and each clover
// block).  FP32 / FP16N: the accumulator is complete here and no memory access moves
// across, so only one direction's neighbour data is live; that keeps the stage
// kernels at 104-109 VGPRs with every complex multiply-add a fused chain (1308 VALU
// instructions per 64 site-RHS in stage 1 against 1608 with sums of products and a
// scheduling barrier alone; 128 RHS: stage 1 / stage 2 6.55 / 8.49 ms against 6.67 /
// 8.96).  FP64 keeps the scheduling barrier and sums of products.
template <class R>
__device__ __forceinline__ void phase_fence(cplx<R> (&a)[12]) {
    if constexpr (sizeof(R) == 4) {
        asm volatile("" : "+v"(a[0].re), "+v"(a[0].im), "+v"(a[1].re), "+v"(a[1].im), "+v"(a[2].re), "+v"(a[2].im),
                     "+v"(a[3].re), "+v"(a[3].im), "+v"(a[4].re), "+v"(a[4].im), "+v"(a[5].re), "+v"(a[5].im)::"memory");
        asm volatile("" : "+v"(a[6].re), "+v"(a[6].im), "+v"(a[7].re), "+v"(a[7].im), "+v"(a[8].re), "+v"(a[8].im),
                     "+v"(a[9].re), "+v"(a[9].im), "+v"(a[10].re), "+v"(a[10].im), "+v"(a[11].re), "+v"(a[11].im)::"memory");
    } else {
        hop_fence();
    }
}

// One work item: the 4 * RW right-hand sides of a tile on kLdsSites sites.
template <class P, int RW, bool DAG, bool CLOVER, bool PRE, int POST, int RED>
__device__ __forceinline__ void stage_lds_body(const StageArgs &A, int sb, int tile) {
    using R = typename P::real;
    constexpr int NT = 4 * RW;
    __shared__ R lnk[8][18][kLdsSites];
    __shared__ int nbr[8][kLdsSites];
    const Geom &g = A.g;
    const int p = A.out_parity;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int h = sb * kLdsSites + lane;
    const bool valid = h < g.vh && in_window(A.win, h, g.vh);
    // ---- phase 1: neighbours and links of the 64 sites (wave w: hops 2w, 2w+1 = mu w fwd / bwd)
    {
        int x = 0, y = 0, z = 0, t = 0;
        if (valid) site_coords(g, p, h, x, y, z, t);
        const int mu = wave;   // wave-uniform; no dynamic indexing of local arrays
#pragma unroll
        for (int fb = 0; fb < 2; ++fb) {
            const int hop = 2 * mu + fb;
            const int d = fb == 0 ? 1 : -1;
            int nx = x, ny = y, nz = z, nt = t;
            bool wrap = false;
            if (mu == 0) {
                nx = x + d;
                if (nx == g.lx) { nx = 0; wrap = true; }
                if (nx < 0) { nx = g.lx - 1; wrap = true; }
            } else if (mu == 1) {
                ny = y + d;
                if (ny == g.ly) { ny = 0; wrap = true; }
                if (ny < 0) { ny = g.ly - 1; wrap = true; }
            } else if (mu == 2) {
                nz = z + d;
                if (nz == g.lz) { nz = 0; wrap = true; }
                if (nz < 0) { nz = g.lz - 1; wrap = true; }
            } else {
                nt = t + d;
                if (nt == g.lt) { nt = 0; wrap = true; }
                if (nt < 0) { nt = g.lt - 1; wrap = true; }
            }
            const R eta = (mu == 3 && wrap && g.antiperiodic) ? R(-1) : R(1);
            const int hn = valid ? cb_index(g, nx, ny, nz, nt) : 0;
            cplx<R> L[9];
            if (valid) {
                GaugeIO<P>::load(A.gp, fb == 0 ? p : 1 - p, mu, g.vh, fb == 0 ? h : hn, L);
            } else {
#pragma unroll
                for (int k = 0; k < 9; ++k) L[k] = {R(0), R(0)};
            }
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    // forward: L[a][b]; backward: (L^dagger)[a][b] = conj(L[b][a])
                    const cplx<R> e = fb == 0 ? L[a * 3 + b] : conj(L[b * 3 + a]);
                    lnk[hop][2 * (a * 3 + b)][lane] = eta * e.re;
                    lnk[hop][2 * (a * 3 + b) + 1][lane] = eta * e.im;
                }
            nbr[hop][lane] = hn;
        }
    }
    __syncthreads();
    // ---- phase 2: one RHS per wave per round
    // RED: 0 none, 1 <w, out>, 2 <out, y> and |out|^2, 3 |out|^2; FP64 modes: 4 |v - A out|^2
    // (v the clover input), 5 out = a y + b H in - A y2 with |out|^2, 6 the hop input is an
    // FP32 half-vector (no reduction), 7 y2 is an FP32 half-vector, added to w as well, with
    // |out|^2
    constexpr int NQ = RED == 1 ? 2 : (RED == 2 ? 3 : (RED == 6 ? 0 : (RED >= 3 ? 1 : 0)));
    constexpr bool WIDEN_IN = RED == 6, WIDEN_Y2 = RED == 7;
    static_assert(RED != 4 || (CLOVER && POST == 0 && sizeof(R) == 8), "reduction 4: FP64 clover stages");
    static_assert(RED != 5 || (!CLOVER && POST == 2 && sizeof(R) == 8), "reduction 5: FP64 residual stages");
    static_assert(RED < 6 || (sizeof(R) == 8 && (RED == 6 ? POST == 0 : POST == 2)), "modes 6, 7: FP64 stages");
#pragma unroll 1
    for (int rw = 0; rw < RW; ++rw) {
        const int slot = A.tile_slots[tile * NT + rw * 4 + wave];
        if (slot < 0) continue;   // wave-uniform
        if (A.flag_filter && !(A.st[slot].flag != 0 && A.st[slot].status == LAPH_RHS_ACTIVE)) continue;
        double part[NQ > 0 ? NQ : 1];
#pragma unroll
        for (int q = 0; q < (NQ > 0 ? NQ : 1); ++q) part[q] = 0.0;
        if (valid) {
            cplx<R> acc[12];
#pragma unroll
            for (int c = 0; c < 12; ++c) acc[c] = {R(0), R(0)};
            const char *src = A.in.at(slot);
            // a scheduling fence per direction: the loads of a direction's forward and
            // backward hops overlap (3 % faster than a fence per hop, 1.5 % faster than
            // none), while the loads of later directions stay after its products
            lds_hop<P, 0, DAG, true, WIDEN_IN>(src, g.vh, lnk, nbr, lane, A.one, acc);
            lds_hop<P, 0, DAG, false, WIDEN_IN>(src, g.vh, lnk, nbr, lane, A.one, acc);
            phase_fence(acc);
            lds_hop<P, 1, DAG, true, WIDEN_IN>(src, g.vh, lnk, nbr, lane, A.one, acc);
            lds_hop<P, 1, DAG, false, WIDEN_IN>(src, g.vh, lnk, nbr, lane, A.one, acc);
            phase_fence(acc);
            lds_hop<P, 2, DAG, true, WIDEN_IN>(src, g.vh, lnk, nbr, lane, A.one, acc);
            lds_hop<P, 2, DAG, false, WIDEN_IN>(src, g.vh, lnk, nbr, lane, A.one, acc);
            phase_fence(acc);
            lds_hop<P, 3, DAG, true, WIDEN_IN>(src, g.vh, lnk, nbr, lane, A.one, acc);
            lds_hop<P, 3, DAG, false, WIDEN_IN>(src, g.vh, lnk, nbr, lane, A.one, acc);
            phase_fence(acc);
            if (PRE) {
                cplx<R> zz[12];
                SpinorIO<P>::load(A.z.at(slot), g.vh, h, zz);
                const R cz = R(A.c);
#pragma unroll
                for (int c = 0; c < 12; ++c) acc[c] = acc[c] + cz * zz[c];
            }
            R n2res = R(0);   // reduction 4
            if (CLOVER) {
                const char *cl = A.clover + (size_t)A.tile_mass[tile] * A.clover_mass_stride;
#pragma unroll
                for (int blk = 0; blk < 2; ++blk) {
                    R m[36];
                    CloverIO<P>::load(cl, blk, g.vh, h, m);
                    cplx<R> o[6];
                    if constexpr (sizeof(R) == 4)
                        herm6_apply_fma(m, &acc[6 * blk], o);
                    else
                        herm6_apply(m, &acc[6 * blk], o);
                    if constexpr (RED == 4) {
                        // this block of v = b (c z + H in) and of the output b A^-1 (c z + H in),
                        // then |v - A out|^2 with the clover term A = (4 + m0) + C of the output
                        // parity: the residual of a half reconstructed as out = A^-1 v
                        // an opaque site index keeps the term's loads inside the RHS loop
                        int ht = h;
                        asm volatile("" : "+v"(ht));
                        R mt[36];
                        CloverIO<F64>::load(A.clover_term, blk, g.vh, ht, mt);
                        const R bv = R(A.b), dg = R(A.diag[A.tile_mass[tile]]);
                        cplx<R> vb[6], ob[6], q[6];
#pragma unroll
                        for (int i = 0; i < 6; ++i) {
                            vb[i] = bv * acc[6 * blk + i];
                            ob[i] = bv * o[i];
                        }
                        herm6_apply(mt, ob, q, dg);
#pragma unroll
                        for (int i = 0; i < 6; ++i) {
                            const cplx<R> d = vb[i] - q[i];
                            n2res += d.re * d.re + d.im * d.im;
                        }
                    }
#pragma unroll
                    for (int i = 0; i < 6; ++i) acc[6 * blk + i] = o[i];
                    phase_fence(acc);
                }
            }
            cplx<R> res[12], yy[12];
            const R bb = R(A.b);
#pragma unroll
            for (int c = 0; c < 12; ++c) res[c] = bb * acc[c];
            if (POST >= 1) {
                SpinorIO<P>::load(A.y.at(slot), g.vh, h, yy);
                const R aa = R(A.a);
#pragma unroll
                for (int c = 0; c < 12; ++c) res[c] = res[c] + aa * yy[c];
            }
            if constexpr (RED == 5) {
                // res -= A y2, the clover term A = (4 + m0) + C of the output parity, one
                // chiral block at a time (with the reduction: y - D y2 of the full operator)
                int ht = h;
                asm volatile("" : "+v"(ht));
                const R dg = R(A.diag[A.tile_mass[tile]]);
#pragma unroll
                for (int blk = 0; blk < 2; ++blk) {
                    cplx<R> y2[6], q[6];
                    R mt[36];
                    SpinorIO<P>::load_block(A.y2.at(slot), g.vh, ht, blk, y2);
                    CloverIO<F64>::load(A.clover_term, blk, g.vh, ht, mt);
                    herm6_apply(mt, y2, q, dg);
#pragma unroll
                    for (int i = 0; i < 6; ++i) res[6 * blk + i] = res[6 * blk + i] - q[i];
                }
            } else if (POST >= 2) {
                cplx<R> y2[12];
                if constexpr (WIDEN_Y2) {
                    cplx<float> yf[12];
                    SpinorIO<F32>::load(A.y2.at(slot), g.vh, h, yf);
#pragma unroll
                    for (int c = 0; c < 12; ++c) y2[c] = {R(yf[c].re), R(yf[c].im)};
                } else {
                    SpinorIO<P>::load(A.y2.at(slot), g.vh, h, y2);
                }
                const R aa2 = R(A.a2);
#pragma unroll
                for (int c = 0; c < 12; ++c) res[c] = res[c] + aa2 * y2[c];
            }
            SpinorIO<P>::store(A.out.at(slot), g.vh, h, res);
            hop_fence();
            if constexpr (WIDEN_Y2) {
                // fold the correction y2 into x64 (w) as well (no other site reads w here);
                // y2 is loaded again (a cache hit) rather than kept live across the store
                int hw = h;
                asm volatile("" : "+v"(hw));
                cplx<float> yf[12];
                cplx<R> xw[12];
                SpinorIO<F32>::load(A.y2.at(slot), g.vh, hw, yf);
                SpinorIO<P>::load(A.w.at(slot), g.vh, hw, xw);
#pragma unroll
                for (int c = 0; c < 12; ++c) xw[c] = xw[c] + cplx<R>{R(yf[c].re), R(yf[c].im)};
                SpinorIO<P>::store(A.w.at(slot), g.vh, hw, xw);
            }
            if (RED == 1) {
                cplx<R> ww[12];
                SpinorIO<P>::load(A.w.at(slot), g.vh, h, ww);
                cplx<R> d = {R(0), R(0)};
#pragma unroll
                for (int c = 0; c < 12; ++c) cmac_conj(d, ww[c], res[c]);
                part[0] = d.re;
                part[1] = d.im;
            } else if (RED == 2) {
                cplx<R> d = {R(0), R(0)};
                R n2 = R(0);
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    cmac_conj(d, res[c], yy[c]);
                    n2 += res[c].re * res[c].re + res[c].im * res[c].im;
                }
                part[0] = d.re;
                part[1] = d.im;
                part[2] = n2;
            } else if (RED == 3 || RED == 5 || RED == 7) {
                R n2 = R(0);
#pragma unroll
                for (int c = 0; c < 12; ++c) n2 += res[c].re * res[c].re + res[c].im * res[c].im;
                part[0] = n2;
            } else if (RED == 4) {
                part[0] = n2res;
            }
        }
        if constexpr (NQ > 0) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                double s = part[q];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
                if (lane == 0) A.partials[((size_t)slot * 3 + q) * A.pstride + sb] = s;
            }
        }
    }
}

template <class P, int RW, bool DAG, bool CLOVER, bool PRE, int POST, int RED>
__global__ __launch_bounds__(256) void stage_lds_kernel(StageArgs A) {
    const int nt = *A.ntiles;
    int first, end, step;
    stage_item_range(nt * A.nsb, A.dispatch_order, first, end, step);
    for (int w = first; w < end; w += step) {
        int sb, tile;
        stage_item(w, A.site_major, A.nsb, nt, sb, tile);
        sb = tiled_block(sb, A.nyb, A.tz, A.tt, A.g.lz);
        if (block_outside(A.win, sb * kLdsSites, min(kLdsSites, A.g.vh - sb * kLdsSites), A.g.vh)) continue;
        stage_lds_body<P, RW, DAG, CLOVER, PRE, POST, RED>(A, sb, tile);
        __syncthreads();   // the next item stages its links in the same LDS
    }
}

// ---------------------------------------------------------------------------
// dispatch (FP32 / FP16N; instantiated in dslash_f32.hip and dslash_f16.hip)
// ---------------------------------------------------------------------------
template <class P, int RW, bool DAG, bool CLOVER, bool PRE, int POST, int RED>
inline void launch_lds_t(const StageArgs &a, hipStream_t st) {
    const int nblk = stage_grid(a.nsb * a.ntiles_max, a.grid_cap);
    hipLaunchKernelGGL((stage_lds_kernel<P, RW, DAG, CLOVER, PRE, POST, RED>), dim3(nblk), dim3(256), 0, st, a);
}

template <class P, int RW, bool DAG>
inline bool launch_lds_combo(const StageSpec &s, const StageArgs &a, hipStream_t st) {
    constexpr bool is64 = std::is_same<P, F64>::value;
    // masked (reliable-update) stages exist in FP64 only; the kernel skips unflagged slots
    if (s.flagged && !is64) return false;
    const int key = s.clover * 1000 + s.pre * 100 + s.post * 10 + s.red;
    switch (key) {
        case 0: launch_lds_t<P, RW, DAG, false, false, 0, 0>(a, st); return true;       // bare hop
        case 1000: launch_lds_t<P, RW, DAG, true, false, 0, 0>(a, st); return true;    // A^-1 H in
        case 1011: launch_lds_t<P, RW, DAG, true, false, 1, 1>(a, st); return true;    // v = p - A^-1 H t, <r^, v>
        case 1012: launch_lds_t<P, RW, DAG, true, false, 1, 2>(a, st); return true;    // t = s - A^-1 H t, <t,s>,|t|^2
        default: break;
    }
    if constexpr (is64) {
        switch (key) {
            case 10: launch_lds_t<P, RW, DAG, false, false, 1, 0>(a, st); return true;     // y + b H in
            case 13: launch_lds_t<P, RW, DAG, false, false, 1, 3>(a, st); return true;     // residual part
            case 1023: launch_lds_t<P, RW, DAG, true, false, 2, 3>(a, st); return true;    // r64, |r64|^2
            case 1100: launch_lds_t<P, RW, DAG, true, true, 0, 0>(a, st); return true;     // A^-1 (c z + H in)
            case 1104: launch_lds_t<P, RW, DAG, true, true, 0, 4>(a, st); return true;     // same, |v - A out|^2
            case 25: launch_lds_t<P, RW, DAG, false, false, 2, 5>(a, st); return true;      // a y + b H in - A y2
            case 1006: launch_lds_t<P, RW, DAG, true, false, 0, 6>(a, st); return true;    // A^-1 H in, in FP32
            case 1027: launch_lds_t<P, RW, DAG, true, false, 2, 7>(a, st); return true;    // r64, y2 FP32, w += y2
            default: break;
        }
    }
    return false;
}

template <class P>
inline bool launch_lds_p(const StageSpec &s, const StageArgs &a, hipStream_t st) {
    const bool d = s.dagger != 0;
    switch (s.tiles.nr) {
        case 4: return d ? launch_lds_combo<P, 1, true>(s, a, st) : launch_lds_combo<P, 1, false>(s, a, st);
        case 8: return d ? launch_lds_combo<P, 2, true>(s, a, st) : launch_lds_combo<P, 2, false>(s, a, st);
        case 16: return d ? launch_lds_combo<P, 4, true>(s, a, st) : launch_lds_combo<P, 4, false>(s, a, st);
        default: return false;
    }
}

bool launch_stage_lds_f64(const StageSpec &s, const StageArgs &a, hipStream_t st);
bool launch_stage_lds_f32(const StageSpec &s, const StageArgs &a, hipStream_t st);
bool launch_stage_lds_f16(const StageSpec &s, const StageArgs &a, hipStream_t st);

}  // namespace laph
