// Fused BLAS-1 kernels of the batched BiCGStab, their FP64 partial reductions,
// and the per-slot finalize kernels that turn the partials into the solver's
// scalars on the device (no host round trip inside an iteration).
//
// Every vector kernel runs on a 2-D grid (site block, entry of the slot list)
// and touches each site once; inner products are accumulated per site in the
// kernel's arithmetic precision, per thread block in FP64 (wave shuffles, then
// LDS) and across blocks by the finalize kernels in a fixed order, so results
// are reproducible run to run.
#include "laph_blas.h"

namespace laph {

constexpr int kB = 256;

__device__ __forceinline__ void reduce_store(double *v, int nv, double *dst, size_t q_stride) {
    __shared__ double red[kB / 64][4];
    for (int q = 0; q < nv; ++q) {
        double s = v[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        v[q] = s;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int q = 0; q < nv; ++q) red[wave][q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int q = 0; q < nv; ++q) {
            double s = 0;
            for (int w = 0; w < kB / 64; ++w) s += red[w][q];
            dst[q * q_stride] = s;
        }
    // a block handles several slots in turn: red is written again next round
    __syncthreads();
}

// Entries of the slot list this launch walks: the flagged list (built on the
// device after the rho finalize) in flagged mode, the slot list otherwise.
__device__ __forceinline__ int blas_count(const BlasArgs &A, int mode) {
    return mode == kModeFlagged ? *A.nflist : *A.nlist;
}

// slot of list entry j, or -1 if it has nothing to do in this mode
__device__ __forceinline__ int blas_slot_at(const BlasArgs &A, int mode, int j) {
    const int s = mode == kModeFlagged ? A.flist[j] : A.list[j];
    const SlotState &st = A.st[s];
    if (mode == kModeActive && st.status != LAPH_RHS_ACTIVE) return -1;
    if (mode == kModeFlagged && !(st.status == LAPH_RHS_ACTIVE && st.flag != 0)) return -1;
    return s;
}

// Grid rows walk the list entries j = blockIdx.y, blockIdx.y + gridDim.y, ...;
// the slot test is uniform over the block.
#define LAPH_FOR_SLOTS(A, mode, s)                                                              \
    for (int j_ = blockIdx.y, n_ = blas_count(A, mode); j_ < n_; j_ += gridDim.y)              \
        if (const int s = blas_slot_at(A, mode, j_); s >= 0)

template <class R>
__device__ __forceinline__ cplx<R> c_of(double2 z) {
    return {R(z.x), R(z.y)};
}

// p = r + beta (p - omega v);  beta == 0 means p = r (fresh start: p, v not read)
template <class P>
__global__ __launch_bounds__(kB) void p_update_kernel(BlasArgs A) {
    using R = typename P::real;
    const int h = blockIdx.x * kB + threadIdx.x;
    if (h >= A.vh) return;
    LAPH_FOR_SLOTS(A, kModeActive, s) {
        const double2 beta = A.st[s].beta;
        cplx<R> r[12];
        SpinorIO<P>::load(A.r.at(s), A.vh, h, r);
        if (beta.x == 0.0 && beta.y == 0.0) {
            SpinorIO<P>::store(A.p.at(s), A.vh, h, r);
            continue;
        }
        const cplx<R> b = c_of<R>(beta), w = c_of<R>(A.st[s].omega);
        cplx<R> p[12], v[12];
        SpinorIO<P>::load(A.p.at(s), A.vh, h, p);
        SpinorIO<P>::load(A.v.at(s), A.vh, h, v);
#pragma unroll
        for (int c = 0; c < 12; ++c) p[c] = r[c] + b * (p[c] - w * v[c]);
        SpinorIO<P>::store(A.p.at(s), A.vh, h, p);
    }
}

// r = r - alpha v   (r becomes s)
template <class P>
__global__ __launch_bounds__(kB) void s_update_kernel(BlasArgs A) {
    using R = typename P::real;
    const int h = blockIdx.x * kB + threadIdx.x;
    if (h >= A.vh) return;
    LAPH_FOR_SLOTS(A, kModeActive, s) {
        const cplx<R> al = c_of<R>(A.st[s].alpha);
        cplx<R> r[12], v[12];
        SpinorIO<P>::load(A.r.at(s), A.vh, h, r);
        SpinorIO<P>::load(A.v.at(s), A.vh, h, v);
#pragma unroll
        for (int c = 0; c < 12; ++c) r[c] = r[c] - al * v[c];
        SpinorIO<P>::store(A.r.at(s), A.vh, h, r);
    }
}

// x_lo += alpha p + omega s (x_lo = ... after a fold or at the start);  r = s - omega t;
// partials <r^, r>, |r|^2
template <class P, class PX>
__global__ __launch_bounds__(kB) void xr_update_kernel(BlasArgs A) {
    using R = typename P::real;
    using RX = typename PX::real;
    const int h = blockIdx.x * kB + threadIdx.x;
    LAPH_FOR_SLOTS(A, kModeActive, s) {
        double part[3] = {0, 0, 0};
        if (h < A.vh) {
            const cplx<R> al = c_of<R>(A.st[s].alpha), om = c_of<R>(A.st[s].omega);
            cplx<R> p[12], r[12], t[12], rh[12];
            cplx<RX> x[12];
            SpinorIO<P>::load(A.p.at(s), A.vh, h, p);
            SpinorIO<P>::load(A.r.at(s), A.vh, h, r);
            SpinorIO<P>::load(A.t.at(s), A.vh, h, t);
            if (A.st[s].xlo_zero) {
#pragma unroll
                for (int c = 0; c < 12; ++c) x[c] = {RX(0), RX(0)};
            } else {
                SpinorIO<PX>::load(A.x.at(s), A.vh, h, x);
            }
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                cplx<R> dx = al * p[c] + om * r[c];
                x[c] = x[c] + cplx<RX>{RX(dx.re), RX(dx.im)};
                r[c] = r[c] - om * t[c];
            }
            SpinorIO<PX>::store(A.x.at(s), A.vh, h, x);
            SpinorIO<P>::store(A.r.at(s), A.vh, h, r);
            SpinorIO<P>::load(A.rh.at(s), A.vh, h, rh);
            cplx<R> d = {R(0), R(0)};
            R n2 = R(0);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                cmac_conj(d, rh[c], r[c]);
                n2 += r[c].re * r[c].re + r[c].im * r[c].im;
            }
            part[0] = d.re;
            part[1] = d.im;
            part[2] = n2;
        }
        reduce_store(part, 3, A.partials + (size_t)s * 3 * A.pstride + blockIdx.x, A.pstride);
    }
}

// reliable update, part 1: x64 += x_lo (flagged slots).  x_lo is not cleared here: the
// update's finalize marks it zero (xlo_zero) and the next x/r update overwrites it.
template <class PX>
__global__ __launch_bounds__(kB) void accumulate_kernel(BlasArgs A, int mode) {
    using RX = typename PX::real;
    const int h = blockIdx.x * kB + threadIdx.x;
    if (h >= A.vh) return;
    LAPH_FOR_SLOTS(A, mode, s) {
        if (A.st[s].xlo_zero) continue;   // uniform: nothing to fold
        cplx<RX> x[12];
        cplx<double> y[12];
        SpinorIO<PX>::load(A.x.at(s), A.vh, h, x);
        SpinorIO<F64>::load(A.x64.at(s), A.vh, h, y);
#pragma unroll
        for (int c = 0; c < 12; ++c) y[c] = y[c] + cplx<double>{(double)x[c].re, (double)x[c].im};
        SpinorIO<F64>::store(A.x64.at(s), A.vh, h, y);
    }
}

// r = lo(r64); restart (flag 2) or init: r^ = r (the init finalize marks x_lo zero).
// partials <r^, r>, |r|^2
template <class P, class PX>
__global__ __launch_bounds__(kB) void lower_kernel(BlasArgs A, int mode, int init) {
    using R = typename P::real;
    const int h = blockIdx.x * kB + threadIdx.x;
    LAPH_FOR_SLOTS(A, mode, s) {
        double part[3] = {0, 0, 0};
        if (h < A.vh) {
            cplx<double> y[12];
            SpinorIO<F64>::load(A.r64.at(s), A.vh, h, y);
            cplx<R> r[12], rh[12];
#pragma unroll
            for (int c = 0; c < 12; ++c) r[c] = {R(y[c].re), R(y[c].im)};
            SpinorIO<P>::store(A.r.at(s), A.vh, h, r);
            // work with the stored (rounded) values so r^ and r agree exactly
            SpinorIO<P>::load(A.r.at(s), A.vh, h, r);
            const bool reset = init || A.st[s].flag == 2;
            if (reset) {
                SpinorIO<P>::store(A.rh.at(s), A.vh, h, r);
                SpinorIO<P>::load(A.rh.at(s), A.vh, h, rh);
            } else {
                SpinorIO<P>::load(A.rh.at(s), A.vh, h, rh);
            }
            cplx<R> d = {R(0), R(0)};
            R n2 = R(0);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                cmac_conj(d, rh[c], r[c]);
                n2 += r[c].re * r[c].re + r[c].im * r[c].im;
            }
            part[0] = d.re;
            part[1] = d.im;
            part[2] = n2;
        }
        reduce_store(part, 3, A.partials + (size_t)s * 3 * A.pstride + blockIdx.x, A.pstride);
    }
}

// |v|^2 of one or two FP64 half-vectors per slot (partials q = 0); sites outside
// the window are not read (the vectors are zero there)
__global__ __launch_bounds__(kB) void norm2_kernel(BlasArgs A, Operand v1, Operand v2, int mode) {
    const int h = blockIdx.x * kB + threadIdx.x;
    const bool live = h < A.vh && in_window(A.win, h, A.vh);
    LAPH_FOR_SLOTS(A, mode, s) {
        double part[1] = {0};
        if (live) {
            cplx<double> y[12];
            SpinorIO<F64>::load(v1.at(s), A.vh, h, y);
            double n2 = 0;
#pragma unroll
            for (int c = 0; c < 12; ++c) n2 += y[c].re * y[c].re + y[c].im * y[c].im;
            if (v2.base) {
                SpinorIO<F64>::load(v2.at(s), A.vh, h, y);
#pragma unroll
                for (int c = 0; c < 12; ++c) n2 += y[c].re * y[c].re + y[c].im * y[c].im;
            }
            part[0] = n2;
        }
        reduce_store(part, 1, A.partials + (size_t)s * 3 * A.pstride + blockIdx.x, A.pstride);
    }
}

// dst = src (FP64 half-vectors) per slot; outside the window src is zero and not read
__global__ __launch_bounds__(kB) void copy64_kernel(BlasArgs A, Operand dst, Operand src, int mode) {
    const int h = blockIdx.x * kB + threadIdx.x;
    if (h >= A.vh) return;
    const bool live = in_window(A.win, h, A.vh);
    LAPH_FOR_SLOTS(A, mode, s) {
        cplx<double> y[12];
        if (live) {
            SpinorIO<F64>::load(src.at(s), A.vh, h, y);
        } else {
#pragma unroll
            for (int c = 0; c < 12; ++c) y[c] = {0.0, 0.0};
        }
        SpinorIO<F64>::store(dst.at(s), A.vh, h, y);
    }
}

// Flagged slots after the rho finalize: the list of slots that take a reliable
// update this iteration, and FP64 register tiles of them (tiles never mix
// masses).  One block; entries of the static FP64 tile table (already grouped
// by mass) are tested in parallel, then packed in table order by one thread.
__global__ __launch_bounds__(kB) void flag_tiles_kernel(FlagArgs A) {
    __shared__ int ks[kB], km[kB];
    const int total = *A.ntiles * A.nr;
    int cur = -1, fill = 0, cm = -1, nf = 0;   // packing state (thread 0)
    for (int base = 0; base < total; base += kB) {
        const int e = base + (int)threadIdx.x;
        int s = -1, m = 0;
        if (e < total) {
            s = A.tile_slots[e];
            m = A.tile_mass[e / A.nr];
            if (s >= 0 && !(A.st[s].status == LAPH_RHS_ACTIVE && A.st[s].flag != 0)) s = -1;
        }
        ks[threadIdx.x] = s;
        km[threadIdx.x] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            const int n = min(kB, total - base);
            for (int i = 0; i < n; ++i) {
                const int si = ks[i];
                if (si < 0) continue;
                if (cur < 0 || fill == A.nr || km[i] != cm) {
                    ++cur;
                    for (int k = 0; k < A.nr; ++k) A.out_slots[cur * A.nr + k] = -1;
                    A.out_mass[cur] = km[i];
                    cm = km[i];
                    fill = 0;
                }
                A.out_slots[cur * A.nr + fill++] = si;
                A.flist[nf++] = si;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *A.out_ntiles = cur + 1;
        *A.nflist = nf;
    }
}

// ---------------------------------------------------------------------------
// finalize kernels: one 64-thread wave per slot sums the partials in fixed order
// ---------------------------------------------------------------------------
// Eight independent loads in flight per lane: the partials were just written by
// workgroups on every XCD, and a loop that waits for each load in turn spends ~0.1 ms
// of latency per slot and quantity.  The summation order is still fixed.
__device__ __forceinline__ double wave_sum_partials(const double *p, int nsb) {
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int i = threadIdx.x;
    for (; i + 7 * 64 < nsb; i += 8 * 64) {
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] += p[i + 64 * k];
    }
    for (; i < nsb; i += 64) a[0] += p[i];
    double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    return s;
}

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ bool finite2(double2 a) { return isfinite(a.x) && isfinite(a.y); }
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

__global__ void finalize_kernel(FinArgs A, int what) {
    const int j = blockIdx.x;
    if (j >= *A.nlist) return;
    const int s = A.list[j];
    SlotState &st = A.st[s];
    const double *P = A.partials + (size_t)s * 3 * A.pstride;
    const bool active = st.status == LAPH_RHS_ACTIVE;
    switch (what) {
        case kFinAlpha: {  // sigma = <r^, v>; alpha = rho / sigma
            if (!active) return;
            const double2 sig = make_double2(wave_sum_partials(P, A.nsb), wave_sum_partials(P + A.pstride, A.nsb));
            if (threadIdx.x) return;
            if (!finite2(sig) || cabs2(sig) <= 1e-300 * (cabs2(st.rho) + 1e-300) || cabs2(sig) == 0.0) {
                st.alpha = make_double2(0, 0);
                st.flag = 2;
            } else {
                st.alpha = cdiv(st.rho, sig);
            }
            return;
        }
        case kFinOmega: {  // omega = <t, s> / |t|^2
            if (!active) return;
            const double2 ts = make_double2(wave_sum_partials(P, A.nsb), wave_sum_partials(P + A.pstride, A.nsb));
            const double tt = wave_sum_partials(P + 2 * A.pstride, A.nsb);
            if (threadIdx.x) return;
            if (!(tt > 0) || !isfinite(tt) || !finite2(ts)) {
                st.omega = make_double2(0, 0);
                st.flag = 2;
            } else {
                st.omega = make_double2(ts.x / tt, ts.y / tt);
            }
            return;
        }
        case kFinRho: {  // rho_new = <r^, r>, r2 = |r|^2; beta; decide on a reliable update
            if (!active) return;
            const double2 rn = make_double2(wave_sum_partials(P, A.nsb), wave_sum_partials(P + A.pstride, A.nsb));
            const double r2 = wave_sum_partials(P + 2 * A.pstride, A.nsb);
            if (threadIdx.x) return;
            st.iters += 1;
            st.r2 = r2;
            if (!isfinite(r2) || !finite2(rn)) st.flag = 2;
            if (st.flag != 2) {
                if (cabs2(st.omega) == 0.0 || cabs2(st.rho) == 0.0 || cabs2(rn) == 0.0) {
                    st.flag = 2;
                } else {
                    st.beta = cmul(cdiv(rn, st.rho), cdiv(st.alpha, st.omega));
                }
            }
            st.rho_prev = st.rho;
            st.rho = rn;
            st.xlo_zero = 0;   // the x/r update just wrote x_lo
            if (r2 <= st.stop2 || r2 < st.delta2 * st.r2_upd || st.iters >= st.maxiter) st.flag |= 1;
            return;
        }
        case kFinUpdate: {  // r2_upd = |b_hat - M x64|^2 after a reliable update
            if (!(active && st.flag != 0)) return;
            const double r2 = wave_sum_partials(P, A.nsb);
            if (threadIdx.x) return;
            st.updates += 1;
            st.r2_upd = r2;
            st.xlo_zero = 1;   // folded into x64 by this update (accumulate, or the FP64 stage forming r64)
            if (!isfinite(r2)) {
                st.status = LAPH_RHS_NONFINITE;
            } else if (r2 <= st.stop2) {
                st.status = LAPH_RHS_CONVERGED;
            } else if (st.iters >= st.maxiter) {
                st.status = LAPH_RHS_NOCONV;
            } else if (st.flag == 2) {
                st.restarts += 1;
                if (st.restarts > A.max_restarts) st.status = LAPH_RHS_BREAKDOWN;
            }
            return;
        }
        case kFinRho2:    // after r = lo(r64): rho and beta from the corrected residual
        case kFinInit: {  // first residual of a solve
            const bool init = what == kFinInit;
            if (!(active && (init || st.flag != 0))) return;
            const double2 rn = make_double2(wave_sum_partials(P, A.nsb), wave_sum_partials(P + A.pstride, A.nsb));
            const double r2 = wave_sum_partials(P + 2 * A.pstride, A.nsb);
            if (threadIdx.x) return;
            st.r2 = r2;
            if (init || st.flag == 2) {
                st.beta = make_double2(0, 0);
                st.rho_prev = make_double2(1, 0);
                st.alpha = make_double2(1, 0);
                st.omega = make_double2(1, 0);
            } else {
                st.beta = cmul(cdiv(rn, st.rho_prev), cdiv(st.alpha, st.omega));
            }
            st.rho = rn;
            st.flag = 0;
            if (init) st.xlo_zero = 1;
            return;
        }
        case kFinBnorm: {  // |B|^2 of the full-lattice source; zero or non-finite sources end here
            const double b2 = wave_sum_partials(P, A.nsb);
            if (threadIdx.x) return;
            st.bnorm2 = b2;
            if (!isfinite(b2)) st.status = LAPH_RHS_NONFINITE;
            return;
        }
        case kFinR64: {  // |r64|^2 at the start of a solve pass
            if (!active) return;
            const double r2 = wave_sum_partials(P, A.nsb);
            if (threadIdx.x) return;
            st.r2_upd = r2;
            if (!isfinite(r2)) st.status = LAPH_RHS_NONFINITE;
            else if (r2 <= st.stop2) st.status = LAPH_RHS_CONVERGED;
            return;
        }
        case kFinTrueRes: {  // accumulate |B - D X|^2 (called for the even and the odd part)
            const double r2 = wave_sum_partials(P, A.nsb);
            if (threadIdx.x) return;
            st.true_res2 += r2;
            return;
        }
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <class F>
static laph_status dispatch_prec(int prec, F &&f) {
    if (prec == LAPH_F64) return f(F64{}, F64{});
    if (prec == LAPH_F32) return f(F32{}, F32{});
    return f(F16N{}, F32{});
}

laph_status blas_p_update(const Ctx &c, const BlasArgs &a, int prec) {
    dim3 grid(a.nsb, a.nlist_max);
    return dispatch_prec(prec, [&](auto P, auto) {
        hipLaunchKernelGGL(p_update_kernel<decltype(P)>, grid, dim3(kB), 0, c.stream, a);
        return check_launch("p_update_kernel");
    });
}
laph_status blas_s_update(const Ctx &c, const BlasArgs &a, int prec) {
    dim3 grid(a.nsb, a.nlist_max);
    return dispatch_prec(prec, [&](auto P, auto) {
        hipLaunchKernelGGL(s_update_kernel<decltype(P)>, grid, dim3(kB), 0, c.stream, a);
        return check_launch("s_update_kernel");
    });
}
laph_status blas_xr_update(const Ctx &c, const BlasArgs &a, int prec) {
    dim3 grid(a.nsb, a.nlist_max);
    return dispatch_prec(prec, [&](auto P, auto PX) {
        hipLaunchKernelGGL((xr_update_kernel<decltype(P), decltype(PX)>), grid, dim3(kB), 0, c.stream, a);
        return check_launch("xr_update_kernel");
    });
}
// grid rows: one per list entry, or a quarter of them in flagged mode (a block
// then walks several flagged slots; the flagged count is known only on the device)
static dim3 blas_grid(const BlasArgs &a, int mode) {
    const int rows = mode == kModeFlagged ? (a.nlist_max + 3) / 4 : a.nlist_max;
    return dim3(a.nsb, rows > 0 ? rows : 1);
}

laph_status blas_accumulate(const Ctx &c, const BlasArgs &a, int prec, int mode) {
    dim3 grid = blas_grid(a, mode);
    return dispatch_prec(prec, [&](auto, auto PX) {
        hipLaunchKernelGGL(accumulate_kernel<decltype(PX)>, grid, dim3(kB), 0, c.stream, a, mode);
        return check_launch("accumulate_kernel");
    });
}
laph_status blas_lower(const Ctx &c, const BlasArgs &a, int prec, int mode, int init) {
    dim3 grid = blas_grid(a, mode);
    return dispatch_prec(prec, [&](auto P, auto PX) {
        hipLaunchKernelGGL((lower_kernel<decltype(P), decltype(PX)>), grid, dim3(kB), 0, c.stream, a, mode, init);
        return check_launch("lower_kernel");
    });
}
laph_status blas_norm2(const Ctx &c, const BlasArgs &a, Operand v1, Operand v2, int mode) {
    dim3 grid = blas_grid(a, mode);
    hipLaunchKernelGGL(norm2_kernel, grid, dim3(kB), 0, c.stream, a, v1, v2, mode);
    return check_launch("norm2_kernel");
}
laph_status blas_copy64(const Ctx &c, const BlasArgs &a, Operand dst, Operand src, int mode) {
    dim3 grid = blas_grid(a, mode);
    hipLaunchKernelGGL(copy64_kernel, grid, dim3(kB), 0, c.stream, a, dst, src, mode);
    return check_launch("copy64_kernel");
}
laph_status blas_flag_tiles(const Ctx &c, const FlagArgs &f) {
    hipLaunchKernelGGL(flag_tiles_kernel, dim3(1), dim3(kB), 0, c.stream, f);
    return check_launch("flag_tiles_kernel");
}
laph_status blas_finalize(const Ctx &c, const FinArgs &f, int what) {
    hipLaunchKernelGGL(finalize_kernel, dim3(f.nlist_max), dim3(64), 0, c.stream, f, what);
    return check_launch("finalize_kernel");
}

}  // namespace laph
