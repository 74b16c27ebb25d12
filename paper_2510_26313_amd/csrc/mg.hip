// Two-level aggregation multigrid for the Wilson-clover matrix D(m0).
//
// The paper's production solver is an adaptive geometric multigrid (Sec. "QUDA":
// the workhorse of the Dirac-matrix solves; Sec. "Performance Measurement
// Method": a mixed-precision multigrid solve is the kernel of the computation),
// and batching is motivated partly by the small parallelism of its coarse grids
// (Sec. "Batched Linear Solves").  The method, in the aggregation form used here:
//
//  * near-null vectors: caller-given start vectors relaxed by inverse iteration
//    with the library's batched FP32-inner solver (x <- D^-1 x);
//  * prolongator P: on each aggregate (a block of fine sites) and chirality
//    (spins 0,1 / 2,3; gamma5 = diag(1,1,-1,-1)) the restricted halves of the
//    vectors, Gram-Schmidt orthonormalised in order; restriction R = P^dagger;
//  * coarse matrix D_c = P^dagger D P, a 9-point stencil of (2 nv x 2 nv) blocks
//    on the coarse lattice, built on the GPU in FP64;
//  * one cycle per outer iteration (all in FP32 on the fine grid): pre-smoother,
//    restrict the residual, coarse BiCGStab, prolong, post-smoother.  The
//    smoother solves D e = r approximately through the even-odd Schur system:
//    b^ from r, a few minimal-residual steps on M^ e_e = b^, then the odd
//    half e_o = A_oo^-1 (r_o + 1/2 H_oe e_e).  After it the odd residual is zero
//    and the even one is A_ee times the MR residual;
//  * outer flexible GCR(m) in mixed precision: x, r, b in FP64; search directions
//    z_k = K r and w_k = D z_k in FP32; every m steps (and at the end) the residual
//    is recomputed in FP64 (the reliable update), so the FP32 directions never
//    limit the attainable accuracy.
//
// All right-hand sides of a call are batched: every kernel takes the RHS as a grid
// dimension, every scalar is per RHS on the device, and converged RHS are frozen.
#include <algorithm>
#include <cmath>
#include <vector>

#include "dslash_kernels.h"
#include "laph_mg.h"
#include "laph_reduce.h"
#include "laph_solver.h"

namespace laph {

namespace {

constexpr int kMB = 256;          // threads of the multigrid kernels
constexpr int kMgBlasBlocks = 1024;   // grid-stride cap of the fine-vector reductions

struct MgDev {
    int bx, by, bz, bt;
    int xc, yc, zc, tc;
    int nc, asize, nv, ncv;
};

MgDev mg_dev(const MgGeom &g) {
    MgDev m;
    m.bx = g.block[0];
    m.by = g.block[1];
    m.bz = g.block[2];
    m.bt = g.block[3];
    m.xc = g.cdim[0];
    m.yc = g.cdim[1];
    m.zc = g.cdim[2];
    m.tc = g.cdim[3];
    m.nc = g.nc;
    m.asize = g.asize;
    m.nv = g.nv;
    m.ncv = g.ncv;
    return m;
}

__device__ __forceinline__ int agg_of(const MgDev &m, int x, int y, int z, int t) {
    return (((t / m.bt) * m.zc + z / m.bz) * m.yc + y / m.by) * m.xc + x / m.bx;
}

// fine coordinates of site k (x fastest) of aggregate a
__device__ __forceinline__ void agg_site(const MgDev &m, int a, int k, int &x, int &y, int &z, int &t) {
    const int ax = a % m.xc;
    int r = a / m.xc;
    const int ay = r % m.yc;
    r /= m.yc;
    const int az = r % m.zc;
    const int at = r / m.zc;
    const int kx = k % m.bx;
    int q = k / m.bx;
    const int ky = q % m.by;
    q /= m.by;
    const int kz = q % m.bz;
    const int kt = q / m.bz;
    x = ax * m.bx + kx;
    y = ay * m.by + ky;
    z = az * m.bz + kz;
    t = at * m.bt + kt;
}

// coarse neighbour of a in direction d (0 self, 1 + 2 mu forward, 2 + 2 mu backward)
__device__ __forceinline__ int coarse_nbr(const MgDev &m, int a, int d) {
    if (d == 0) return a;
    const int mu = (d - 1) >> 1;
    const int k = (d & 1) ? 1 : -1;
    int c[4] = {a % m.xc, (a / m.xc) % m.yc, (a / (m.xc * m.yc)) % m.zc, a / (m.xc * m.yc * m.zc)};
    const int ext[4] = {m.xc, m.yc, m.zc, m.tc};
    c[mu] = (c[mu] + k + ext[mu]) % ext[mu];
    return ((c[3] * m.zc + c[2]) * m.yc + c[1]) * m.xc + c[0];
}

// Sum of N doubles per thread over a kMB-thread block, fixed order; the result is
// returned to every thread.  red: LDS scratch of (kMB / 64) * N doubles.
template <int N>
__device__ __forceinline__ void block_sum_bcast(double (&v)[N], double *red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < N; ++q) {
        double s = v[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        v[q] = s;
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < N; ++q) red[wave * N + q] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < N; ++q) {
        double s = 0;
        for (int w = 0; w < kMB / 64; ++w) s += red[w * N + q];
        v[q] = s;
    }
    __syncthreads();
}

// Wave reduction of N values per lane (N a power of two, <= 64) that leaves lane l
// with the wave's sum of v[l % N]: a transposing butterfly inside groups of N lanes
// (each step a lane keeps half of its values and adds its partner's matching half,
// N - 1 exchanges instead of log2(64) per value), then plain steps add the 64 / N groups.
template <int N>
__device__ __forceinline__ double wave_transpose_sum(double (&v)[N], int lane) {
#pragma unroll
    for (int o = N / 2; o >= 1; o >>= 1) {
        const bool up = (lane & o) != 0;
#pragma unroll
        for (int i = 0; i < o; ++i) {
            const double send = up ? v[i] : v[i + o];
            const double keep = up ? v[i + o] : v[i];
            v[i] = keep + __shfl_xor(send, o, 64);
        }
    }
    double s = v[0];
#pragma unroll
    for (int o = 32; o >= N; o >>= 1) s += __shfl_xor(s, o, 64);
    return s;
}

__device__ __forceinline__ double2 ld2(const char *hv, int vh, int c, int h) {
    return reinterpret_cast<const double2 *>(hv)[(size_t)c * vh + h];
}
__device__ __forceinline__ void st2(char *hv, int vh, int c, int h, double2 v) {
    reinterpret_cast<double2 *>(hv)[(size_t)c * vh + h] = v;
}

// ---------------------------------------------------------------------------
// setup kernels
// ---------------------------------------------------------------------------

// Gram-Schmidt of the nv basis vectors on one (aggregate, chirality): grid (nc, 2).
__global__ __launch_bounds__(kMB) void mg_orth_kernel(Geom g, MgDev m, char *basis, size_t bstride, size_t half,
                                                      int *flag) {
    __shared__ double red[(kMB / 64) * 2];
    const int a = blockIdx.x, chi = blockIdx.y;
    const int c0 = 6 * chi;
    for (int i = 0; i < m.nv; ++i) {
        char *wi = basis + (size_t)i * bstride;
        double n0[2] = {0, 0};
        for (int k = threadIdx.x; k < m.asize; k += kMB) {
            int x, y, z, t;
            agg_site(m, a, k, x, y, z, t);
            const int p = (x + y + z + t) & 1, h = cb_index(g, x, y, z, t);
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const double2 v = ld2(wi + p * half, g.vh, c0 + c, h);
                n0[0] += v.x * v.x + v.y * v.y;
            }
        }
        block_sum_bcast<2>(n0, red);
        for (int j = 0; j < i; ++j) {
            const char *wj = basis + (size_t)j * bstride;
            double d[2] = {0, 0};
            for (int k = threadIdx.x; k < m.asize; k += kMB) {
                int x, y, z, t;
                agg_site(m, a, k, x, y, z, t);
                const int p = (x + y + z + t) & 1, h = cb_index(g, x, y, z, t);
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    const double2 u = ld2(wj + p * half, g.vh, c0 + c, h), v = ld2(wi + p * half, g.vh, c0 + c, h);
                    d[0] += u.x * v.x + u.y * v.y;   // conj(u) v
                    d[1] += u.x * v.y - u.y * v.x;
                }
            }
            block_sum_bcast<2>(d, red);
            for (int k = threadIdx.x; k < m.asize; k += kMB) {
                int x, y, z, t;
                agg_site(m, a, k, x, y, z, t);
                const int p = (x + y + z + t) & 1, h = cb_index(g, x, y, z, t);
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    const double2 u = ld2(wj + p * half, g.vh, c0 + c, h);
                    double2 v = ld2(wi + p * half, g.vh, c0 + c, h);
                    v.x -= d[0] * u.x - d[1] * u.y;
                    v.y -= d[0] * u.y + d[1] * u.x;
                    st2(wi + p * half, g.vh, c0 + c, h, v);
                }
            }
        }
        double n2[2] = {0, 0};
        for (int k = threadIdx.x; k < m.asize; k += kMB) {
            int x, y, z, t;
            agg_site(m, a, k, x, y, z, t);
            const int p = (x + y + z + t) & 1, h = cb_index(g, x, y, z, t);
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const double2 v = ld2(wi + p * half, g.vh, c0 + c, h);
                n2[0] += v.x * v.x + v.y * v.y;
            }
        }
        block_sum_bcast<2>(n2, red);
        // a half in the span of the earlier ones (relative to its own size) fails the setup
        if (!(n2[0] > 1e-24 * n0[0]) || !(n2[0] > 0)) {
            if (threadIdx.x == 0) flag[0] = 1;
            return;
        }
        const double s = 1.0 / sqrt(n2[0]);
        for (int k = threadIdx.x; k < m.asize; k += kMB) {
            int x, y, z, t;
            agg_site(m, a, k, x, y, z, t);
            const int p = (x + y + z + t) & 1, h = cb_index(g, x, y, z, t);
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                double2 v = ld2(wi + p * half, g.vh, c0 + c, h);
                v.x *= s;
                v.y *= s;
                st2(wi + p * half, g.vh, c0 + c, h, v);
            }
        }
        __syncthreads();
    }
}

// basis vector j at one fine site, keeping only the components of chirality chi
__device__ __forceinline__ void load_chiral(const char *bj, size_t half, int vh, int p, int h, int chi,
                                            cplx<double> (&v)[12]) {
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        if ((c / 6) == chi) {
            const double2 u = ld2(bj + p * half, vh, c, h);
            v[c] = {u.x, u.y};
        } else {
            v[c] = {0.0, 0.0};
        }
    }
}

// y += -1/2 eta (1 - gamma_mu) U_mu(x) v(x + mu)  (FWD) or
// y += -1/2 eta (1 + gamma_mu) U_mu(x - mu)^dagger v(x - mu)
template <int MU, bool FWD>
__device__ __forceinline__ void coarse_hop(const Geom &g, const GaugePtrs &gp, const char *bj, size_t half, int chi,
                                           const int (&xs)[4], int p, int h, cplx<double> (&y)[12]) {
    constexpr int S = FWD ? -1 : 1;
    const int ext = MU == 0 ? g.lx : (MU == 1 ? g.ly : (MU == 2 ? g.lz : g.lt));
    int n[4] = {xs[0], xs[1], xs[2], xs[3]};
    bool wrap = false;
    if (FWD) {
        n[MU] = xs[MU] + 1;
        if (n[MU] == ext) { n[MU] = 0; wrap = true; }
    } else {
        n[MU] = xs[MU] - 1;
        if (n[MU] < 0) { n[MU] = ext - 1; wrap = true; }
    }
    const double eta = (MU == 3 && wrap && g.antiperiodic) ? -1.0 : 1.0;
    const int hn = cb_index(g, n[0], n[1], n[2], n[3]);
    cplx<double> v[12], hs[6], u[6], L[9];
    load_chiral(bj, half, g.vh, 1 - p, hn, chi, v);
    if (FWD)
        GaugeIO<F64>::load(gp, p, MU, g.vh, h, L);
    else
        GaugeIO<F64>::load(gp, 1 - p, MU, g.vh, hn, L);
    spin_project<MU, S>(v, hs);
    colour_mul<!FWD>(L, hs, u);
    spin_accumulate<MU, S>(y, u, -0.5 * eta);
}

// Compiler barrier of the coarse build: y is complete here and no memory access moves
// across, so the loads of one hop direction are live at a time (without it the kernel
// kept every direction's link and neighbour in flight: 492 VGPRs and spills).
__device__ __forceinline__ void build_fence(cplx<double> (&y)[12]) {
    asm volatile("" : "+v"(y[0].re), "+v"(y[0].im), "+v"(y[1].re), "+v"(y[1].im), "+v"(y[2].re), "+v"(y[2].im),
                 "+v"(y[3].re), "+v"(y[3].im), "+v"(y[4].re), "+v"(y[4].im), "+v"(y[5].re), "+v"(y[5].im)::"memory");
    asm volatile("" : "+v"(y[6].re), "+v"(y[6].im), "+v"(y[7].re), "+v"(y[7].im), "+v"(y[8].re), "+v"(y[8].im),
                 "+v"(y[9].re), "+v"(y[9].im), "+v"(y[10].re), "+v"(y[10].im), "+v"(y[11].re), "+v"(y[11].im)::"memory");
}

template <int MU>
__device__ __forceinline__ void coarse_dir(const Geom &g, const GaugePtrs &gp, const MgDev &m, const char *bj,
                                           size_t half, int chi, const int (&xs)[4], int p, int h, int d,
                                           cplx<double> (&y)[12]) {
    const int b = MU == 0 ? m.bx : (MU == 1 ? m.by : (MU == 2 ? m.bz : m.bt));
    const bool cross_f = (xs[MU] % b) == b - 1, cross_b = (xs[MU] % b) == 0;
    if ((d == 0 && !cross_f) || (d == 1 + 2 * MU && cross_f)) coarse_hop<MU, true>(g, gp, bj, half, chi, xs, p, h, y);
    build_fence(y);
    if ((d == 0 && !cross_b) || (d == 2 + 2 * MU && cross_b)) coarse_hop<MU, false>(g, gp, bj, half, chi, xs, p, h, y);
}

// Aggregate-major copy of the basis for the coarse build:
// wagg[((a nv + i) 12 + c) asize + k] = component c of w_i at site k of aggregate a, so that
// the build's dot products read each (i, c) as one contiguous row across the aggregate's
// threads (the field layout scatters an aggregate's sites over many cache lines).
// Grid (nc, nv); one thread per site of the aggregate (asize <= kMB).
__global__ __launch_bounds__(kMB) void mg_agg_pack_kernel(Geom g, MgDev m, const char *basis, size_t bstride,
                                                          size_t half, double2 *wagg) {
    const int a = blockIdx.x, i = blockIdx.y, k = threadIdx.x;
    if (k >= m.asize) return;
    int x, y, z, t;
    agg_site(m, a, k, x, y, z, t);
    const int p = (x + y + z + t) & 1;
    const int h = cb_index(g, x, y, z, t);
    const char *bi = basis + (size_t)i * bstride + p * half;
    double2 *out = wagg + ((size_t)a * m.nv + i) * 12 * m.asize + k;
#pragma unroll
    for (int c = 0; c < 12; ++c) out[(size_t)c * m.asize] = ld2(bi, g.vh, c, h);
}

// D_c[a][d][(chi, i)][(chi', j)] = sum_{x in a} <w_(chi,i)(x), (D^(d) P_chi' w_j)(x)>, where D^(0)
// holds the clover term and the hops inside the aggregate and D^(d) (d > 0) the hop
// that leaves it in direction d.  Grid nc; one thread per fine site (asize <= kMB).
__global__ __launch_bounds__(kMB) void mg_coarse_build_kernel(Geom g, GaugePtrs gp, MgDev m, const char *basis,
                                                              size_t bstride, size_t half, const double2 *wagg,
                                                              const char *cterm0, const char *cterm1,
                                                              const double *diag, int mass, double2 *C) {
    __shared__ double red[(kMB / 64) * 4 * kMgMaxVec];
    const int a = blockIdx.x;
    const int k = threadIdx.x;
    const bool own = k < m.asize;
    int xs[4] = {0, 0, 0, 0}, p = 0, h = 0;
    if (own) {
        agg_site(m, a, k, xs[0], xs[1], xs[2], xs[3]);
        p = (xs[0] + xs[1] + xs[2] + xs[3]) & 1;
        h = cb_index(g, xs[0], xs[1], xs[2], xs[3]);
    }
    const double dg = diag[mass];
#pragma unroll 1
    for (int j = 0; j < m.nv; ++j) {
        const char *bj = basis + (size_t)j * bstride;
#pragma unroll 1
        for (int chi2 = 0; chi2 < 2; ++chi2) {
#pragma unroll 1
            for (int d = 0; d < 9; ++d) {
                // the site's coordinates are opaque per iteration: the neighbour and link
                // addresses derived from them are recomputed here instead of being hoisted
                // out of the loops and held in registers (hundreds of VGPRs)
                asm volatile("" : "+v"(h), "+v"(p), "+v"(xs[0]), "+v"(xs[1]), "+v"(xs[2]), "+v"(xs[3]));
                cplx<double> y[12];
#pragma unroll
                for (int c = 0; c < 12; ++c) y[c] = {0.0, 0.0};
                if (own) {
                    if (d == 0) {
                        cplx<double> v[12];
                        load_chiral(bj, half, g.vh, p, h, chi2, v);
                        double mm[36];
                        CloverIO<F64>::load(p == 0 ? cterm0 : cterm1, chi2, g.vh, h, mm);
                        // constant offsets keep v and y in registers
                        if (chi2 == 0)
                            herm6_apply(mm, &v[0], &y[0], dg);
                        else
                            herm6_apply(mm, &v[6], &y[6], dg);
                    }
                    build_fence(y);
                    coarse_dir<0>(g, gp, m, bj, half, chi2, xs, p, h, d, y);
                    build_fence(y);
                    coarse_dir<1>(g, gp, m, bj, half, chi2, xs, p, h, d, y);
                    build_fence(y);
                    coarse_dir<2>(g, gp, m, bj, half, chi2, xs, p, h, d, y);
                    build_fence(y);
                    coarse_dir<3>(g, gp, m, bj, half, chi2, xs, p, h, d, y);
                    build_fence(y);
                }
                // dots with every basis vector i, both chiralities, four vectors at a time
                // (16 values [i][chi][re, im] per lane keep the register count low): lane
                // q < 16 of every wave holds its wave's sum of value q, thread q adds the
                // four waves in order
                const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
                const double2 *wa = wagg + (size_t)a * m.nv * 12 * m.asize + k;
#pragma unroll 1
                for (int i0 = 0; i0 < m.nv; i0 += 4) {
                    double acc[16];
#pragma unroll
                    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
                    if (own) {
#pragma unroll
                        for (int ii = 0; ii < 4; ++ii) {
                            if (i0 + ii < m.nv) {
#pragma unroll
                                for (int c = 0; c < 12; ++c) {
                                    const double2 w = wa[((size_t)(i0 + ii) * 12 + c) * m.asize];
                                    const int q = 4 * ii + 2 * (c / 6);
                                    acc[q] += w.x * y[c].re + w.y * y[c].im;
                                    acc[q + 1] += w.x * y[c].im - w.y * y[c].re;
                                }
                            }
                            // one basis vector's loads in flight at a time
                            asm volatile("" : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]),
                                         "+v"(acc[5]), "+v"(acc[6]), "+v"(acc[7])::"memory");
                            asm volatile("" : "+v"(acc[8]), "+v"(acc[9]), "+v"(acc[10]), "+v"(acc[11]),
                                         "+v"(acc[12]), "+v"(acc[13]), "+v"(acc[14]), "+v"(acc[15])::"memory");
                        }
                    }
                    red[wave * 64 + lane] = wave_transpose_sum<16>(acc, lane);
                    __syncthreads();
                    if (threadIdx.x < 16 && i0 + (threadIdx.x >> 2) < m.nv) {
                        const int q = threadIdx.x, i = i0 + (q >> 2), chi = (q >> 1) & 1;
                        double sum = 0;
                        for (int wv = 0; wv < kMB / 64; ++wv) sum += red[wv * 64 + q];
                        const size_t row = (size_t)chi * m.nv + i, col = (size_t)chi2 * m.nv + j;
                        reinterpret_cast<double *>(C)[((((size_t)a * 9 + d) * m.ncv + row) * m.ncv + col) * 2 +
                                                      (q & 1)] = sum;
                    }
                    __syncthreads();
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// restriction / prolongation
// ---------------------------------------------------------------------------

// out[r][a][(chi, i)] = sum over the sites of a (of the parities in pmask) of
// <w_(chi, i), f_r>.  Grid (nc, n).
template <class P>
__global__ __launch_bounds__(kMB) void mg_restrict_kernel(Geom g, MgDev m, const char *basis, size_t bstride,
                                                          size_t bhalf, Operand f, size_t fhalf, int pmask,
                                                          double2 *out) {
    __shared__ double red[(kMB / 64) * 4 * kMgMaxVec];
    const int a = blockIdx.x, r = blockIdx.y;
    double acc[4 * kMgMaxVec];
#pragma unroll
    for (int q = 0; q < 4 * kMgMaxVec; ++q) acc[q] = 0.0;
    for (int k = threadIdx.x; k < m.asize; k += kMB) {
        int x, y, z, t;
        agg_site(m, a, k, x, y, z, t);
        const int p = (x + y + z + t) & 1;
        if (!((pmask >> p) & 1)) continue;
        const int h = cb_index(g, x, y, z, t);
        cplx<typename P::real> fv[12];
        SpinorIO<P>::load(f.at(r) + p * fhalf, g.vh, h, fv);
#pragma unroll
        for (int i = 0; i < kMgMaxVec; ++i) {
            if (i < m.nv) {
                const char *bi = basis + (size_t)i * bstride + p * bhalf;
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    const double2 w = ld2(bi, g.vh, c, h);
                    const double fr = fv[c].re, fi = fv[c].im;
                    const int q = 4 * i + 2 * (c / 6);
                    acc[q] += w.x * fr + w.y * fi;
                    acc[q + 1] += w.x * fi - w.y * fr;
                }
            }
        }
    }
    block_sum_bcast<4 * kMgMaxVec>(acc, red);
    if (threadIdx.x < m.ncv) {
        const int chi = threadIdx.x / m.nv, i = threadIdx.x % m.nv;
        out[((size_t)r * m.nc + a) * m.ncv + threadIdx.x] = make_double2(acc[4 * i + 2 * chi], acc[4 * i + 2 * chi + 1]);
    }
}

// f_r (+)= P c_r on both parities.  Grid (ceil(2 vh / kMB), n).
template <class P, bool ACC>
__global__ __launch_bounds__(kMB) void mg_prolong_kernel(Geom g, MgDev m, const char *basis, size_t bstride,
                                                         size_t bhalf, const double2 *cv, Operand f, size_t fhalf) {
    using R = typename P::real;
    const int s = blockIdx.x * kMB + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= 2 * g.vh) return;
    const int p = s >= g.vh ? 1 : 0;
    const int h = s - p * g.vh;
    int x, y, z, t;
    site_coords(g, p, h, x, y, z, t);
    const int a = agg_of(m, x, y, z, t);
    const double2 *ca = cv + ((size_t)r * m.nc + a) * m.ncv;
    double re[12], im[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) re[c] = im[c] = 0.0;
    for (int i = 0; i < m.nv; ++i) {
        const double2 c0 = ca[i], c1 = ca[m.nv + i];
        const char *bi = basis + (size_t)i * bstride + p * bhalf;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const double2 w = ld2(bi, g.vh, c, h);
            const double2 cc = c < 6 ? c0 : c1;
            re[c] += cc.x * w.x - cc.y * w.y;
            im[c] += cc.x * w.y + cc.y * w.x;
        }
    }
    char *hv = f.at(r) + p * fhalf;
    cplx<R> o[12];
    if (ACC) SpinorIO<P>::load(hv, g.vh, h, o);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const R pr = R(re[c]), pi = R(im[c]);
        o[c] = ACC ? cplx<R>{o[c].re + pr, o[c].im + pi} : cplx<R>{pr, pi};
    }
    SpinorIO<P>::store(hv, g.vh, h, o);
}

// The cycle's restriction and prolongation: FP32 fields, the FP32 copy of the basis,
// kMgRhsGroup RHS per workgroup (each basis vector is read once per group).
constexpr int kMgRhsGroup = 4;

// out[r][a][(chi, i)] = sum over the sites of a of the parities in pmask of <w_(chi,i), f_r>,
// for the group's RHS.  Grid (nc, ceil(n / kMgRhsGroup)); one site per thread (asize <= kMB).
__global__ __launch_bounds__(kMB) void mg_restrict32_kernel(Geom g, MgDev m, const char *basis, size_t bstride,
                                                            size_t bhalf, Operand f, size_t fhalf, int pmask, int n,
                                                            double2 *out) {
    __shared__ double red[(kMB / 64) * 4 * kMgRhsGroup];
    const int a = blockIdx.x, r0 = blockIdx.y * kMgRhsGroup;
    const int k = threadIdx.x;
    int x = 0, y = 0, z = 0, t = 0;
    bool own = k < m.asize;
    if (own) agg_site(m, a, k, x, y, z, t);
    const int p = (x + y + z + t) & 1;
    own = own && ((pmask >> p) & 1);
    const int h = own ? cb_index(g, x, y, z, t) : 0;
    cplx<float> fv[kMgRhsGroup][12];
#pragma unroll
    for (int rr = 0; rr < kMgRhsGroup; ++rr) {
        if (own && r0 + rr < n) {
            SpinorIO<F32>::load(f.at(r0 + rr) + p * fhalf, g.vh, h, fv[rr]);
        } else {
#pragma unroll
            for (int c = 0; c < 12; ++c) fv[rr][c] = {0.f, 0.f};
        }
    }
    for (int i = 0; i < m.nv; ++i) {
        double acc[4 * kMgRhsGroup];
#pragma unroll
        for (int q = 0; q < 4 * kMgRhsGroup; ++q) acc[q] = 0.0;
        if (own) {
            cplx<float> b[12];
            SpinorIO<F32>::load(basis + (size_t)i * bstride + p * bhalf, g.vh, h, b);
#pragma unroll
            for (int rr = 0; rr < kMgRhsGroup; ++rr)
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    const int q = 4 * rr + 2 * (c / 6);
                    acc[q] += (double)(b[c].re * fv[rr][c].re + b[c].im * fv[rr][c].im);
                    acc[q + 1] += (double)(b[c].re * fv[rr][c].im - b[c].im * fv[rr][c].re);
                }
        }
        block_sum_bcast<4 * kMgRhsGroup>(acc, red);
        if (threadIdx.x < 2 * kMgRhsGroup) {
            const int rr = threadIdx.x >> 1, chi = threadIdx.x & 1;
            if (r0 + rr < n)
                out[((size_t)(r0 + rr) * m.nc + a) * m.ncv + chi * m.nv + i] =
                    make_double2(acc[4 * rr + 2 * chi], acc[4 * rr + 2 * chi + 1]);
        }
    }
}

// f_r (+)= P c_r on both parities for the group's RHS.  Grid (ceil(2 vh / kMB), ceil(n / kMgRhsGroup)).
template <bool ACC>
__global__ __launch_bounds__(kMB) void mg_prolong32_kernel(Geom g, MgDev m, const char *basis, size_t bstride,
                                                           size_t bhalf, const double2 *cv, Operand f, size_t fhalf,
                                                           int n) {
    const int s = blockIdx.x * kMB + threadIdx.x;
    const int r0 = blockIdx.y * kMgRhsGroup;
    if (s >= 2 * g.vh) return;
    const int p = s >= g.vh ? 1 : 0;
    const int h = s - p * g.vh;
    int x, y, z, t;
    site_coords(g, p, h, x, y, z, t);
    const int a = agg_of(m, x, y, z, t);
    cplx<float> o[kMgRhsGroup][12];
#pragma unroll
    for (int rr = 0; rr < kMgRhsGroup; ++rr)
#pragma unroll
        for (int c = 0; c < 12; ++c) o[rr][c] = {0.f, 0.f};
    for (int i = 0; i < m.nv; ++i) {
        cplx<float> b[12];
        SpinorIO<F32>::load(basis + (size_t)i * bstride + p * bhalf, g.vh, h, b);
#pragma unroll
        for (int rr = 0; rr < kMgRhsGroup; ++rr) {
            const int r = min(r0 + rr, n - 1);
            const double2 c0 = cv[((size_t)r * m.nc + a) * m.ncv + i], c1 = cv[((size_t)r * m.nc + a) * m.ncv + m.nv + i];
            const float c0r = float(c0.x), c0i = float(c0.y), c1r = float(c1.x), c1i = float(c1.y);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const float cr = c < 6 ? c0r : c1r, ci = c < 6 ? c0i : c1i;
                o[rr][c] = {o[rr][c].re + cr * b[c].re - ci * b[c].im, o[rr][c].im + cr * b[c].im + ci * b[c].re};
            }
        }
    }
#pragma unroll
    for (int rr = 0; rr < kMgRhsGroup; ++rr) {
        if (r0 + rr >= n) break;
        char *hv = f.at(r0 + rr) + p * fhalf;
        if (ACC) {
            cplx<float> prev[12];
            SpinorIO<F32>::load(hv, g.vh, h, prev);
#pragma unroll
            for (int c = 0; c < 12; ++c) o[rr][c] = {o[rr][c].re + prev[c].re, o[rr][c].im + prev[c].im};
        }
        SpinorIO<F32>::store(hv, g.vh, h, o[rr]);
    }
}

// ---------------------------------------------------------------------------
// coarse operator and coarse BiCGStab (FP64, coarse vectors [n][nc][ncv])
// ---------------------------------------------------------------------------
// out_r = D_c in_r.  Grid (nc, RHS groups), kMB threads: for each of the 9 directions the
// block row C[a][d] and the neighbour's coarse vectors of the group's RHS are staged in
// LDS (coalesced), then each thread accumulates up to kCoarsePairs (row, RHS) outputs, so
// every block row is read from memory once per group.
constexpr int kCoarsePairs = 4;
inline int coarse_group(int ncv) { return std::min(64, kCoarsePairs * kMB / ncv); }

__global__ __launch_bounds__(kMB) void mg_coarse_apply_kernel(MgDev m, const double2 *C, const double2 *in,
                                                              double2 *out, int n, int group) {
    extern __shared__ double2 lds[];
    double2 *ct = lds;                                    // ncv x ncv block
    double2 *xt = lds + (size_t)m.ncv * m.ncv;            // group x ncv neighbour vectors
    const int a = blockIdx.x, r0 = blockIdx.y * group;
    const int g = min(group, n - r0);
    const int npair = m.ncv * g, nblk = m.ncv * m.ncv;
    double acc[2 * kCoarsePairs];
#pragma unroll
    for (int k = 0; k < 2 * kCoarsePairs; ++k) acc[k] = 0.0;
    for (int d = 0; d < 9; ++d) {
        const int nb = coarse_nbr(m, a, d);
        __syncthreads();
        const double2 *cb = C + ((size_t)a * 9 + d) * nblk;
        for (int i = threadIdx.x; i < nblk; i += kMB) ct[i] = cb[i];
        for (int i = threadIdx.x; i < npair; i += kMB) {
            const int rl = i / m.ncv, col = i - rl * m.ncv;
            xt[i] = in[((size_t)(r0 + rl) * m.nc + nb) * m.ncv + col];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kCoarsePairs; ++k) {
            const int pidx = threadIdx.x + k * kMB;
            if (pidx < npair) {
                const int rl = pidx / m.ncv, row = pidx - rl * m.ncv;
                const double2 *crow = ct + (size_t)row * m.ncv, *x = xt + (size_t)rl * m.ncv;
                double sr = acc[2 * k], si = acc[2 * k + 1];
                for (int col = 0; col < m.ncv; ++col) {
                    const double2 cc = crow[col], vv = x[col];
                    sr += cc.x * vv.x - cc.y * vv.y;
                    si += cc.x * vv.y + cc.y * vv.x;
                }
                acc[2 * k] = sr;
                acc[2 * k + 1] = si;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kCoarsePairs; ++k) {
        const int pidx = threadIdx.x + k * kMB;
        if (pidx < npair) {
            const int rl = pidx / m.ncv, row = pidx - rl * m.ncv;
            out[((size_t)(r0 + rl) * m.nc + a) * m.ncv + row] = make_double2(acc[2 * k], acc[2 * k + 1]);
        }
    }
}

struct CgState {
    double2 rho, alpha, omega, beta;
    double b2, r2, tol2;
    int done;
};

// partial[(r * 2 + q) * 2 + (re, im)][blk] of <x_q, y_q> over len complex entries
__global__ __launch_bounds__(kMB) void mg_cdot_kernel(const double2 *x0, const double2 *y0, const double2 *x1,
                                                      const double2 *y1, int nq, size_t len, double *partial) {
    __shared__ double red[(kMB / 64) * 4];
    const int r = blockIdx.y;
    double v[4] = {0, 0, 0, 0};
    for (size_t i = (size_t)blockIdx.x * kMB + threadIdx.x; i < len; i += (size_t)gridDim.x * kMB) {
        const size_t o = (size_t)r * len + i;
        const double2 a = x0[o], b = y0[o];
        v[0] += a.x * b.x + a.y * b.y;
        v[1] += a.x * b.y - a.y * b.x;
        if (nq > 1) {
            const double2 c = x1[o], d = y1[o];
            v[2] += c.x * d.x + c.y * d.y;
            v[3] += c.x * d.y - c.y * d.x;
        }
    }
    block_sum_bcast<4>(v, red);
    if (threadIdx.x < 4) partial[((size_t)r * 4 + threadIdx.x) * gridDim.x + blockIdx.x] = v[threadIdx.x];
}

enum { kCgInit, kCgRho, kCgAlpha, kCgOmega, kCgRes };

// Sum the partials of RHS blockIdx.x (fixed order) and advance its BiCGStab scalars.
__global__ __launch_bounds__(kMB) void mg_cscalar_kernel(CgState *st, const double *partial, int nblk, int what,
                                                         double tol) {
    __shared__ double red[(kMB / 64) * 4];
    const int r = blockIdx.x;
    double v[4] = {0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblk; b += kMB)
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] += partial[((size_t)r * 4 + q) * nblk + b];
    block_sum_bcast<4>(v, red);
    if (threadIdx.x != 0) return;
    CgState &s = st[r];
    auto cdiv = [](double2 a, double2 b) {
        const double d = b.x * b.x + b.y * b.y;
        return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
    };
    auto cmul = [](double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); };
    if (what == kCgInit) {   // v0 = <b, b>
        s.b2 = v[0];
        s.r2 = v[0];
        s.tol2 = tol * tol * v[0];
        s.rho = s.alpha = s.omega = make_double2(1.0, 0.0);
        s.beta = make_double2(0.0, 0.0);
        s.done = !(v[0] > 0);
        return;
    }
    if (s.done) return;
    if (what == kCgRho) {   // v0,1 = <r^, r>
        const double2 rn = make_double2(v[0], v[1]);
        if (rn.x == 0 && rn.y == 0) {
            s.done = 1;
            return;
        }
        s.beta = cmul(cdiv(rn, s.rho), cdiv(s.alpha, s.omega));
        s.rho = rn;
    } else if (what == kCgAlpha) {   // v0,1 = <r^, v>
        const double2 sg = make_double2(v[0], v[1]);
        if (sg.x == 0 && sg.y == 0) {
            s.done = 1;
            return;
        }
        s.alpha = cdiv(s.rho, sg);
    } else if (what == kCgOmega) {   // v0,1 = <t, s>, v2 = <t, t>
        // t = 0 means s = 0: omega = 0 still takes x += alpha p and r = s
        s.omega = v[2] > 0 ? make_double2(v[0] / v[2], v[1] / v[2]) : make_double2(0.0, 0.0);
    } else if (what == kCgRes) {   // v0 = <r, r>
        s.r2 = v[0];
        if (v[0] <= s.tol2) s.done = 1;
    }
}

__device__ __forceinline__ double2 cm(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// kind 0: p = r + beta (p - omega v); 1: s = r - alpha v; 2: x += alpha p + omega s, r = s - omega t;
// 3: x = 0, r = r^ = b, p = v = 0
__global__ __launch_bounds__(kMB) void mg_cupdate_kernel(const CgState *st, int kind, size_t len, double2 *x,
                                                         double2 *r, double2 *rh, double2 *p, double2 *v, double2 *s,
                                                         double2 *t, const double2 *b) {
    const int rr = blockIdx.y;
    const CgState &S = st[rr];
    if (kind != 3 && S.done) return;
    for (size_t i = (size_t)blockIdx.x * kMB + threadIdx.x; i < len; i += (size_t)gridDim.x * kMB) {
        const size_t o = (size_t)rr * len + i;
        if (kind == 0) {
            const double2 pv = p[o], vv = v[o], rv = r[o];
            const double2 w = cm(S.omega, vv);
            const double2 q = cm(S.beta, make_double2(pv.x - w.x, pv.y - w.y));
            p[o] = make_double2(rv.x + q.x, rv.y + q.y);
        } else if (kind == 1) {
            const double2 vv = v[o], rv = r[o];
            const double2 w = cm(S.alpha, vv);
            s[o] = make_double2(rv.x - w.x, rv.y - w.y);
        } else if (kind == 2) {
            const double2 ap = cm(S.alpha, p[o]), os = cm(S.omega, s[o]), ot = cm(S.omega, t[o]);
            const double2 xv = x[o], sv = s[o];
            x[o] = make_double2(xv.x + ap.x + os.x, xv.y + ap.y + os.y);
            r[o] = make_double2(sv.x - ot.x, sv.y - ot.y);
        } else {
            const double2 bv = b[o];
            x[o] = make_double2(0.0, 0.0);
            r[o] = bv;
            rh[o] = bv;
            p[o] = make_double2(0.0, 0.0);
            v[o] = make_double2(0.0, 0.0);
        }
    }
}

// ---------------------------------------------------------------------------
// fine-grid vector kernels (full vectors: even half then odd half per RHS)
// ---------------------------------------------------------------------------

// MR step of the smoother (FP32, even half): alpha = <t, rho> / |t|^2 from the stage
// sums; s += alpha rho; rho -= alpha t.  Grid (ceil(vh / kMB), n).
__global__ __launch_bounds__(kMB) void mg_mr_update_kernel(int vh, const double *dots, Operand s, Operand rho,
                                                           Operand t) {
    const int h = blockIdx.x * kMB + threadIdx.x;
    const int r = blockIdx.y;
    if (h >= vh) return;
    const double tt = dots[3 * r + 2];
    const float ar = tt > 0 ? float(dots[3 * r] / tt) : 0.f, ai = tt > 0 ? float(dots[3 * r + 1] / tt) : 0.f;
    cplx<float> sv[12], rv[12], tv[12];
    SpinorIO<F32>::load(s.at(r), vh, h, sv);
    SpinorIO<F32>::load(rho.at(r), vh, h, rv);
    SpinorIO<F32>::load(t.at(r), vh, h, tv);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        sv[c] = {sv[c].re + ar * rv[c].re - ai * rv[c].im, sv[c].im + ar * rv[c].im + ai * rv[c].re};
        rv[c] = {rv[c].re - (ar * tv[c].re - ai * tv[c].im), rv[c].im - (ar * tv[c].im + ai * tv[c].re)};
    }
    SpinorIO<F32>::store(s.at(r), vh, h, sv);
    SpinorIO<F32>::store(rho.at(r), vh, h, rv);
}

// out = x + y on the first np halves (1: the given half only, 2: both) of precision P.
// Grid (ceil(np vh / kMB), n).
template <class P>
__global__ __launch_bounds__(kMB) void mg_add_kernel(int vh, int np, size_t half, Operand out, Operand x, Operand y) {
    const int s = blockIdx.x * kMB + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= np * vh) return;
    const int p = s >= vh ? 1 : 0, h = s - p * vh;
    cplx<typename P::real> a[12], b[12];
    SpinorIO<P>::load(x.at(r) + p * half, vh, h, a);
    SpinorIO<P>::load(y.at(r) + p * half, vh, h, b);
#pragma unroll
    for (int c = 0; c < 12; ++c) a[c] = {a[c].re + b[c].re, a[c].im + b[c].im};
    SpinorIO<P>::store(out.at(r) + p * half, vh, h, a);
}

// zero one half (FP32) of n RHS.  Grid (ceil(vh / kMB), n).
__global__ __launch_bounds__(kMB) void mg_zero_half_kernel(int vh, Operand v) {
    const int h = blockIdx.x * kMB + threadIdx.x;
    if (h >= vh) return;
    cplx<float> z[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) z[c] = {0.f, 0.f};
    SpinorIO<F32>::store(v.at(blockIdx.y), vh, h, z);
}

// out (PO) = in (PI) on full vectors.
template <class PI, class PO>
__global__ __launch_bounds__(kMB) void mg_convert_kernel(int vh, size_t ihalf, size_t ohalf, Operand out, Operand in) {
    const int s = blockIdx.x * kMB + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= 2 * vh) return;
    const int p = s >= vh ? 1 : 0, h = s - p * vh;
    cplx<typename PI::real> a[12];
    cplx<typename PO::real> b[12];
    SpinorIO<PI>::load(in.at(r) + p * ihalf, vh, h, a);
#pragma unroll
    for (int c = 0; c < 12; ++c) b[c] = {typename PO::real(a[c].re), typename PO::real(a[c].im)};
    SpinorIO<PO>::store(out.at(r) + p * ohalf, vh, h, b);
}

struct GcrState {
    double b2, r2, stop2, true_res2;
    double2 gamma;
    double inv;
    int frozen, done, iters, restarts;
};

// partials of <W_q, W_k> (q < k), FP32 vectors.  Grid (nblk, n).
__global__ __launch_bounds__(kMB) void mg_gcr_multidot_kernel(int vh, size_t half, Operand W, int kdim, int k, double *partial,
                                                              const GcrState *gs) {
    __shared__ double red[(kMB / 64) * 2 * kMgMaxRestart];
    const int r = blockIdx.y;
    double acc[2 * kMgMaxRestart];
#pragma unroll
    for (int q = 0; q < 2 * kMgMaxRestart; ++q) acc[q] = 0.0;
    if (!gs[r].frozen) {
        for (int s = blockIdx.x * kMB + threadIdx.x; s < 2 * vh; s += gridDim.x * kMB) {
            const int p = s >= vh ? 1 : 0, h = s - p * vh;
            cplx<float> wk[12];
            SpinorIO<F32>::load(W.at(r * kdim + k) + p * half, vh, h, wk);
#pragma unroll
            for (int q = 0; q < kMgMaxRestart; ++q) {
                if (q < k) {
                    cplx<float> wq[12];
                    SpinorIO<F32>::load(W.at(r * kdim + q) + p * half, vh, h, wq);
#pragma unroll
                    for (int c = 0; c < 12; ++c) {
                        acc[2 * q] += (double)wq[c].re * wk[c].re + (double)wq[c].im * wk[c].im;
                        acc[2 * q + 1] += (double)wq[c].re * wk[c].im - (double)wq[c].im * wk[c].re;
                    }
                }
            }
        }
    }
    block_sum_bcast<2 * kMgMaxRestart>(acc, red);
    if (threadIdx.x < 2 * k) partial[((size_t)r * 2 * kMgMaxRestart + threadIdx.x) * gridDim.x + blockIdx.x] = acc[threadIdx.x];
}

// sums[r][q] = sum over blocks of partial[r][q][.] (nq quantities per RHS, fixed order).  Grid n.
__global__ __launch_bounds__(kMB) void mg_sum_kernel(const double *partial, int nblk, int nq, int qstride, double *sums) {
    const int r = blockIdx.x;
    __shared__ double red[kMB / 64];
    for (int q = 0; q < nq; ++q) {
        double v[1] = {0};
        for (int b = threadIdx.x; b < nblk; b += kMB) v[0] += partial[((size_t)r * qstride + q) * nblk + b];
        block_sum_bcast<1>(v, red);
        if (threadIdx.x == 0) sums[(size_t)r * qstride + q] = v[0];
    }
}

// W_k -= sum_q beta_q W_q, Z_k -= sum_q beta_q Z_q (beta = the sums of the multidot).
__global__ __launch_bounds__(kMB) void mg_gcr_orth_kernel(int vh, size_t half, Operand W, Operand Z, int kdim, int k,
                                                          const double *beta, const GcrState *gs) {
    const int s = blockIdx.x * kMB + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= 2 * vh || gs[r].frozen) return;
    const int p = s >= vh ? 1 : 0, h = s - p * vh;
    const double *bt = beta + (size_t)r * 2 * kMgMaxRestart;
    cplx<float> wk[12], zk[12];
    SpinorIO<F32>::load(W.at(r * kdim + k) + p * half, vh, h, wk);
    SpinorIO<F32>::load(Z.at(r * kdim + k) + p * half, vh, h, zk);
    for (int q = 0; q < k; ++q) {
        const float br = float(bt[2 * q]), bi = float(bt[2 * q + 1]);
        cplx<float> wq[12], zq[12];
        SpinorIO<F32>::load(W.at(r * kdim + q) + p * half, vh, h, wq);
        SpinorIO<F32>::load(Z.at(r * kdim + q) + p * half, vh, h, zq);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            wk[c] = {wk[c].re - (br * wq[c].re - bi * wq[c].im), wk[c].im - (br * wq[c].im + bi * wq[c].re)};
            zk[c] = {zk[c].re - (br * zq[c].re - bi * zq[c].im), zk[c].im - (br * zq[c].im + bi * zq[c].re)};
        }
    }
    SpinorIO<F32>::store(W.at(r * kdim + k) + p * half, vh, h, wk);
    SpinorIO<F32>::store(Z.at(r * kdim + k) + p * half, vh, h, zk);
}

// partials of |W_k|^2 and <W_k, r64>.  Grid (nblk, n); quantities 0: |W|^2, 1, 2: <W, r>.
__global__ __launch_bounds__(kMB) void mg_gcr_dot2_kernel(int vh, size_t half32, size_t half64, Operand W, int kdim, int k,
                                                          Operand r64, double *partial, const GcrState *gs) {
    __shared__ double red[(kMB / 64) * 3];
    const int r = blockIdx.y;
    double v[3] = {0, 0, 0};
    if (!gs[r].frozen) {
        for (int s = blockIdx.x * kMB + threadIdx.x; s < 2 * vh; s += gridDim.x * kMB) {
            const int p = s >= vh ? 1 : 0, h = s - p * vh;
            cplx<float> w[12];
            cplx<double> rr[12];
            SpinorIO<F32>::load(W.at(r * kdim + k) + p * half32, vh, h, w);
            SpinorIO<F64>::load(r64.at(r) + p * half64, vh, h, rr);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const double wr = w[c].re, wi = w[c].im;
                v[0] += wr * wr + wi * wi;
                v[1] += wr * rr[c].re + wi * rr[c].im;
                v[2] += wr * rr[c].im - wi * rr[c].re;
            }
        }
    }
    block_sum_bcast<3>(v, red);
    if (threadIdx.x < 3) partial[((size_t)r * 3 + threadIdx.x) * gridDim.x + blockIdx.x] = v[threadIdx.x];
}

// gamma = <W_k, r> / |W_k|^2, inv = 1 / |W_k| from the sums [r][3].  Grid n, one thread.
__global__ void mg_gcr_scalar_kernel(GcrState *gs, const double *sums, int n) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    GcrState &s = gs[r];
    const double n2 = sums[3 * r];
    if (s.frozen || !(n2 > 0)) {
        s.gamma = make_double2(0.0, 0.0);
        s.inv = 0.0;
        return;
    }
    s.gamma = make_double2(sums[3 * r + 1] / n2, sums[3 * r + 2] / n2);
    s.inv = 1.0 / sqrt(n2);
}

// x += gamma Z_k; r -= gamma W_k; W_k *= inv; Z_k *= inv; partials of |r|^2.  Grid (nblk, n).
__global__ __launch_bounds__(kMB) void mg_gcr_update_kernel(int vh, size_t half32, size_t half64, Operand W,
                                                            Operand Z, int kdim, int k, Operand x64, Operand r64,
                                                            double *partial, const GcrState *gs) {
    __shared__ double red[kMB / 64];
    const int r = blockIdx.y;
    const GcrState &S = gs[r];
    double v[1] = {0};
    for (int s = blockIdx.x * kMB + threadIdx.x; s < 2 * vh; s += gridDim.x * kMB) {
        const int p = s >= vh ? 1 : 0, h = s - p * vh;
        cplx<double> rr[12];
        SpinorIO<F64>::load(r64.at(r) + p * half64, vh, h, rr);
        if (!S.frozen) {
            cplx<float> w[12], z[12];
            cplx<double> xx[12];
            char *wp = W.at(r * kdim + k) + p * half32, *zp = Z.at(r * kdim + k) + p * half32;
            SpinorIO<F32>::load(wp, vh, h, w);
            SpinorIO<F32>::load(zp, vh, h, z);
            SpinorIO<F64>::load(x64.at(r) + p * half64, vh, h, xx);
            const double gr = S.gamma.x, gi = S.gamma.y;
            const float iv = float(S.inv);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const double zr = z[c].re, zi = z[c].im, wr = w[c].re, wi = w[c].im;
                xx[c] = {xx[c].re + gr * zr - gi * zi, xx[c].im + gr * zi + gi * zr};
                rr[c] = {rr[c].re - (gr * wr - gi * wi), rr[c].im - (gr * wi + gi * wr)};
                w[c] = {w[c].re * iv, w[c].im * iv};
                z[c] = {z[c].re * iv, z[c].im * iv};
            }
            SpinorIO<F64>::store(x64.at(r) + p * half64, vh, h, xx);
            SpinorIO<F64>::store(r64.at(r) + p * half64, vh, h, rr);
            SpinorIO<F32>::store(wp, vh, h, w);
            SpinorIO<F32>::store(zp, vh, h, z);
        }
#pragma unroll
        for (int c = 0; c < 12; ++c) v[0] += rr[c].re * rr[c].re + rr[c].im * rr[c].im;
    }
    block_sum_bcast<1>(v, red);
    if (threadIdx.x == 0) partial[(size_t)r * gridDim.x + blockIdx.x] = v[0];
}

// r = b - r (r holds D x on entry), partials of |r|^2 (and of |b|^2 when init).  Grid (nblk, n).
__global__ __launch_bounds__(kMB) void mg_resid_kernel(int vh, size_t half, Operand b, Operand r64, double *partial,
                                                       int with_b) {
    __shared__ double red[(kMB / 64) * 2];
    const int r = blockIdx.y;
    double v[2] = {0, 0};
    for (int s = blockIdx.x * kMB + threadIdx.x; s < 2 * vh; s += gridDim.x * kMB) {
        const int p = s >= vh ? 1 : 0, h = s - p * vh;
        cplx<double> bb[12], rr[12];
        SpinorIO<F64>::load(b.at(r) + p * half, vh, h, bb);
        SpinorIO<F64>::load(r64.at(r) + p * half, vh, h, rr);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            rr[c] = {bb[c].re - rr[c].re, bb[c].im - rr[c].im};
            v[0] += rr[c].re * rr[c].re + rr[c].im * rr[c].im;
            v[1] += bb[c].re * bb[c].re + bb[c].im * bb[c].im;
        }
        SpinorIO<F64>::store(r64.at(r) + p * half, vh, h, rr);
    }
    block_sum_bcast<2>(v, red);
    if (threadIdx.x < 1 + with_b) partial[((size_t)r * 2 + threadIdx.x) * gridDim.x + blockIdx.x] = v[threadIdx.x];
}

// what 0: init (sums [r][2] = |r|^2, |b|^2 with x = 0); 1: after an update (sums [r][1] = |r|^2);
// 2: after a true residual (sums [r][2] = |r|^2).  Grid n, one thread per RHS.
__global__ void mg_gcr_status_kernel(GcrState *gs, const double *sums, int qstride, int n, int what, double tol) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    GcrState &s = gs[r];
    const double r2 = sums[(size_t)r * qstride];
    if (what == 0) {
        s.b2 = sums[(size_t)r * qstride + 1];
        s.stop2 = 0.25 * tol * tol * s.b2;
        s.r2 = r2;
        s.true_res2 = s.b2 > 0 ? r2 / s.b2 : 0.0;
        s.done = s.frozen = !(s.b2 > 0) || s.true_res2 <= tol * tol;
        s.iters = s.restarts = 0;
        return;
    }
    if (what == 1) {
        if (!s.frozen) {
            s.r2 = r2;
            s.iters += 1;
            if (r2 <= s.stop2 || !(r2 == r2)) s.frozen = 1;
        }
        return;
    }
    if (s.done) return;
    s.r2 = r2;
    s.true_res2 = s.b2 > 0 ? r2 / s.b2 : 0.0;
    s.restarts += 1;
    s.done = s.true_res2 <= tol * tol || !(r2 == r2);
    s.frozen = s.done;
}

// tile table of a batch: slots 0 .. n-1 (padded with -1) in tiles of nr, all of one mass
__global__ void mg_tiles_kernel(int *ints, int n, int nr, int ntiles, int mass) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int ns = ntiles * nr;
    if (i < ns)
        ints[i] = i < n ? i : -1;
    else if (i < ns + ntiles)
        ints[i] = mass;
    else if (i == ns + ntiles)
        ints[i] = ntiles;
}

inline dim3 grid2(int items, int n) { return dim3((items + kMB - 1) / kMB, n); }

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

laph_status mg_geometry(const Ctx &c, int nvec, const int block[4], MgGeom &g) {
    if (nvec < 1 || nvec > kMgMaxVec) return set_error(LAPH_ERR_INVALID, "multigrid: nvec must be in 1..%d", kMgMaxVec);
    g.asize = 1;
    for (int i = 0; i < 4; ++i) {
        if (block[i] < 1 || c.dims[i] % block[i])
            return set_error(LAPH_ERR_INVALID, "multigrid: aggregate extent %d = %d does not divide %d", i, block[i],
                             c.dims[i]);
        g.block[i] = block[i];
        g.cdim[i] = c.dims[i] / block[i];
        g.asize *= block[i];
    }
    if (g.asize > kMB) return set_error(LAPH_ERR_INVALID, "multigrid: aggregates of more than %d sites", kMB);
    g.nc = g.cdim[0] * g.cdim[1] * g.cdim[2] * g.cdim[3];
    g.nv = nvec;
    g.ncv = 2 * nvec;
    return LAPH_OK;
}

static size_t full64(const Ctx &c) { return 2 * c.hv(LAPH_F64); }
static size_t full32(const Ctx &c) { return 2 * c.hv(LAPH_F32); }
static size_t coarse_bytes(const MgGeom &g) { return round256((size_t)g.nc * 9 * g.ncv * g.ncv * sizeof(double2)); }

size_t mg_state_bytes(const Ctx &c, const MgGeom &g) {
    return (size_t)g.nv * full64(c) + (size_t)g.nv * full32(c) + coarse_bytes(g) + 256;
}

// The inverse-iteration solves, then (reusing the same bytes) the aggregate-major
// basis copy of the coarse build, nv full fields of FP64.
size_t mg_setup_workspace_bytes(const Ctx &c, const MgGeom &g, int null_passes) {
    const size_t canon = round256((size_t)g.nv * 2 * c.g.vh * 12 * sizeof(double2));
    if (null_passes <= 0) return canon;
    laph_solve_params p;
    laph_default_params(&p);
    p.inner_prec = LAPH_F32;
    p.batched = 1;
    return 2 * canon + solver_workspace_bytes(c, g.nv, p);
}

static laph_status attach(Ctx &c, const MgGeom &g, char *state, size_t bytes, int mass_idx) {
    if (!state || bytes < mg_state_bytes(c, g)) return set_error(LAPH_ERR_WORKSPACE, "multigrid buffer too small");
    MgState &s = c.mgs;
    s.ready = false;
    s.geo = g;
    s.mass_idx = mass_idx;
    s.basis = state;
    s.basis_stride = full64(c);
    s.basis32 = state + (size_t)g.nv * full64(c);
    s.basis32_stride = full32(c);
    s.coarse = reinterpret_cast<double2 *>(state + (size_t)g.nv * (full64(c) + full32(c)));
    s.flag = reinterpret_cast<int *>(state + (size_t)g.nv * (full64(c) + full32(c)) + coarse_bytes(g));
    return LAPH_OK;
}

laph_status mg_setup(Ctx &c, int mass_idx, const MgGeom &g, const double *V0, int null_passes, double null_tol,
                     char *state, size_t state_bytes, char *work, size_t work_bytes) {
    if (mass_idx < 0 || mass_idx >= c.n_mass) return set_error(LAPH_ERR_INVALID, "multigrid: mass index out of range");
    if (work_bytes < mg_setup_workspace_bytes(c, g, null_passes)) return set_error(LAPH_ERR_WORKSPACE, "multigrid setup workspace too small");
    LAPH_TRY(attach(c, g, state, state_bytes, mass_idx));
    MgState &s = c.mgs;
    const double *src = V0;
    if (null_passes > 0) {
        // inverse iteration: x <- D^-1 x with the batched FP32-inner solver (loose tolerance)
        const size_t canon = round256((size_t)g.nv * 2 * c.g.vh * 12 * sizeof(double2));
        double *buf[2] = {reinterpret_cast<double *>(work), reinterpret_cast<double *>(work + canon)};
        laph_solve_params p;
        laph_default_params(&p);
        p.inner_prec = LAPH_F32;
        p.batched = 1;
        p.maxiter = 500;
        Solver solver;
        LAPH_TRY(solver.init(c, g.nv, p, work + 2 * canon, work_bytes - 2 * canon));
        const size_t full = (size_t)2 * c.g.vh * 12;
        std::vector<int> mass(g.nv, mass_idx);
        for (int pass = 0; pass < null_passes; ++pass) {
            SourceSpec sp;
            sp.B = src;
            sp.B_stride = full;
            sp.n = g.nv;
            LAPH_TRY(solver.solve(sp, mass, null_tol, nullptr, full));
            const auto &ws = solver.workspace();
            double *dst = buf[pass & 1];
            LAPH_TRY(unpack_spinor(c, dst, ws.E1, LAPH_F64, g.nv, 0, full));
            LAPH_TRY(unpack_spinor(c, dst, ws.O0, LAPH_F64, g.nv, 1, full));
            int worst = LAPH_OK;
            LAPH_TRY(solver.collect(nullptr, g.nv, null_tol, &worst));   // a loose solve need not converge
            src = dst;
        }
    }
    LAPH_TRY(pack_spinor(c, Operand{s.basis, s.basis_stride}, src, LAPH_F64, g.nv, -1, 0));
    LAPH_HIP(hipMemsetAsync(s.flag, 0, sizeof(int), c.stream));
    const MgDev m = mg_dev(g);
    hipLaunchKernelGGL(mg_orth_kernel, dim3(g.nc, 2), dim3(kMB), 0, c.stream, c.g, m, s.basis, s.basis_stride,
                       c.hv(LAPH_F64), s.flag);
    LAPH_TRY(check_launch("mg_orth_kernel"));
    hipLaunchKernelGGL((mg_convert_kernel<F64, F32>), dim3((2 * c.g.vh + kMB - 1) / kMB, g.nv), dim3(kMB), 0, c.stream,
                       c.g.vh, c.hv(LAPH_F64), c.hv(LAPH_F32), Operand{s.basis32, s.basis32_stride},
                       Operand{s.basis, s.basis_stride});
    LAPH_TRY(check_launch("mg_convert_kernel"));
    // the solves are done: the workspace now holds the aggregate-major basis copy
    double2 *wagg = reinterpret_cast<double2 *>(work);
    hipLaunchKernelGGL(mg_agg_pack_kernel, dim3(g.nc, g.nv), dim3(kMB), 0, c.stream, c.g, m, (const char *)s.basis,
                       s.basis_stride, c.hv(LAPH_F64), wagg);
    LAPH_TRY(check_launch("mg_agg_pack_kernel"));
    hipLaunchKernelGGL(mg_coarse_build_kernel, dim3(g.nc), dim3(kMB), 0, c.stream, c.g, c.gp, m,
                       (const char *)s.basis, s.basis_stride, c.hv(LAPH_F64), (const double2 *)wagg,
                       c.clover_term(0), c.clover_term(1), (const double *)c.mass_diag(), mass_idx, s.coarse);
    LAPH_TRY(check_launch("mg_coarse_build_kernel"));
    int flag = 0;
    LAPH_HIP(hipMemcpyAsync(&flag, s.flag, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    LAPH_HIP(hipStreamSynchronize(c.stream));
    if (flag) return set_error(LAPH_ERR_INVALID, "multigrid: a near-null vector is linearly dependent on an aggregate");
    s.ready = true;
    return LAPH_OK;
}

static laph_status need_mg(const Ctx &c) {
    if (!c.mgs.ready) return set_error(LAPH_ERR_INVALID, "no multigrid set up (laph_mg_setup)");
    return LAPH_OK;
}

laph_status mg_basis_canonical(const Ctx &c, double *out) {
    LAPH_TRY(need_mg(c));
    const MgState &s = c.mgs;
    return unpack_spinor(c, out, Operand{s.basis, s.basis_stride}, LAPH_F64, s.geo.nv, -1, 0);
}

laph_status mg_restrict_canonical(const Ctx &c, double *cvec, const double *f, int n, char *work) {
    LAPH_TRY(need_mg(c));
    const MgState &s = c.mgs;
    const Operand fo{work, full64(c)};
    LAPH_TRY(pack_spinor(c, fo, f, LAPH_F64, n, -1, 0));
    hipLaunchKernelGGL(mg_restrict_kernel<F64>, dim3(s.geo.nc, n), dim3(kMB), 0, c.stream, c.g, mg_dev(s.geo),
                       (const char *)s.basis, s.basis_stride, c.hv(LAPH_F64), fo, c.hv(LAPH_F64), 3,
                       reinterpret_cast<double2 *>(cvec));
    return check_launch("mg_restrict_kernel");
}

laph_status mg_prolong_canonical(const Ctx &c, double *f, const double *cvec, int n, char *work) {
    LAPH_TRY(need_mg(c));
    const MgState &s = c.mgs;
    const Operand fo{work, full64(c)};
    hipLaunchKernelGGL((mg_prolong_kernel<F64, false>), grid2(2 * c.g.vh, n), dim3(kMB), 0, c.stream, c.g,
                       mg_dev(s.geo), (const char *)s.basis, s.basis_stride, c.hv(LAPH_F64),
                       reinterpret_cast<const double2 *>(cvec), fo, c.hv(LAPH_F64));
    LAPH_TRY(check_launch("mg_prolong_kernel"));
    return unpack_spinor(c, f, fo, LAPH_F64, n, -1, 0);
}

static laph_status coarse_apply_dev(const Ctx &c, double2 *out, const double2 *in, int n) {
    const MgState &s = c.mgs;
    const int group = coarse_group(s.geo.ncv);
    const size_t lds = ((size_t)s.geo.ncv * s.geo.ncv + (size_t)group * s.geo.ncv) * sizeof(double2);
    hipLaunchKernelGGL(mg_coarse_apply_kernel, dim3(s.geo.nc, (n + group - 1) / group), dim3(kMB), lds, c.stream,
                       mg_dev(s.geo), (const double2 *)s.coarse, in, out, n, group);
    return check_launch("mg_coarse_apply_kernel");
}

laph_status mg_coarse_apply(const Ctx &c, double *out, const double *in, int n) {
    LAPH_TRY(need_mg(c));
    return coarse_apply_dev(c, reinterpret_cast<double2 *>(out), reinterpret_cast<const double2 *>(in), n);
}

// ---------------------------------------------------------------------------
// the solve
// ---------------------------------------------------------------------------
namespace {

struct MgWs {
    // FP64 full vectors [n]
    Operand b, x, r;
    // FP32 full vectors [n] and [n][kMgMaxRestart]
    Operand Z, W, r32, res, q, hq, sa, sb;
    // coarse vectors [n][nc][ncv]
    double2 *cb, *cx, *cr, *crh, *cp, *cv, *cs, *ct;
    CgState *cst;
    GcrState *gst;
    double *spart;    // stage partials [n][3][pstride]
    double *dots;     // [n][3]
    double *bpart;    // BLAS partials [n][2 kMgMaxRestart][nblk]
    double *sums;     // [n][2 kMgMaxRestart]
    int *tiles;       // stage tile table
};

int mg_tile(int n) { return n >= 16 ? 16 : (n >= 8 ? 8 : 4); }

size_t mg_layout(const Ctx &c, int n, int restart, char *base, MgWs *w) {
    const MgGeom &g = c.mgs.geo;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += round256(bytes);
        return p;
    };
    const size_t f64 = full64(c), f32 = full32(c);
    const size_t cvec = (size_t)g.nc * g.ncv * sizeof(double2);
    MgWs t;
    t.b = Operand{take(n * f64), f64};
    t.x = Operand{take(n * f64), f64};
    t.r = Operand{take(n * f64), f64};
    t.Z = Operand{take((size_t)n * restart * f32), f32};
    t.W = Operand{take((size_t)n * restart * f32), f32};
    t.r32 = Operand{take(n * f32), f32};
    t.res = Operand{take(n * f32), f32};
    t.q = Operand{take(n * f32), f32};
    t.hq = Operand{take(n * f32), f32};
    t.sa = Operand{take(n * f32), f32};
    t.sb = Operand{take(n * f32), f32};
    double2 **cv[8] = {&t.cb, &t.cx, &t.cr, &t.crh, &t.cp, &t.cv, &t.cs, &t.ct};
    for (auto p : cv) *p = reinterpret_cast<double2 *>(take(n * cvec));
    t.cst = reinterpret_cast<CgState *>(take(n * sizeof(CgState)));
    t.gst = reinterpret_cast<GcrState *>(take(n * sizeof(GcrState)));
    t.spart = reinterpret_cast<double *>(take((size_t)n * 3 * partial_stride(c) * sizeof(double)));
    t.dots = reinterpret_cast<double *>(take((size_t)n * 3 * sizeof(double)));
    t.bpart = reinterpret_cast<double *>(take((size_t)n * 2 * kMgMaxRestart * kMgBlasBlocks * sizeof(double)));
    t.sums = reinterpret_cast<double *>(take((size_t)n * 2 * kMgMaxRestart * sizeof(double)));
    const int nr = mg_tile(n);
    t.tiles = reinterpret_cast<int *>(take(((size_t)((n + nr - 1) / nr) * (nr + 1) + 1) * sizeof(int)));
    if (w) *w = t;
    return off;
}

class MgSolver {
   public:
    MgSolver(const Ctx &c, const MgState &run, int n, const MgWs &w) : c(c), n(n), w(w), s(run) {
        nblk = std::min(kMgBlasBlocks, (2 * c.g.vh + kMB - 1) / kMB);
        nr = mg_tile(n);
        ntiles = (n + nr - 1) / nr;
        h32 = c.hv(LAPH_F32);
        h64 = c.hv(LAPH_F64);
        cblk = std::min(256, (int)(((size_t)s.geo.nc * s.geo.ncv + kMB - 1) / kMB));
    }
    laph_status init_tiles();
    laph_status solve(double tol, std::vector<GcrState> &out);
    laph_status component(int what, double *out, const double *in);

   private:
    const Ctx &c;
    int n;
    MgWs w;
    MgState s;   // the attached multigrid with this call's cycle parameters
    int nblk, nr, ntiles, cblk;
    size_t h32, h64;

    Tiles tiles() const {
        Tiles t;
        t.slots = w.tiles;
        t.mass = w.tiles + (size_t)ntiles * nr;
        t.ntiles = w.tiles + (size_t)ntiles * nr + ntiles;
        t.ntiles_max = ntiles;
        t.nr = nr;
        return t;
    }
    static Operand half(Operand v, int p, size_t h) { return Operand{v.base + p * h, v.stride}; }
    Operand sub(Operand v, int k) const { return Operand{v.base + (size_t)k * v.stride, v.stride * s.restart}; }
    // a fused stencil stage on FP32 halves (LDS-staged links), identity tiles
    laph_status stage(int out_parity, Operand in, Operand out, int clover, int post, Operand y, double a, double b,
                      int red, Operand wv) {
        StageSpec st;
        st.prec = LAPH_F32;
        st.form = kFormLds;
        st.site_major = 1;
        st.out_parity = out_parity;
        st.clover = clover;
        st.post = post;
        st.red = red;
        st.in = in;
        st.out = out;
        st.y = y;
        st.w = wv;
        st.a = a;
        st.b = b;
        st.tiles = tiles();
        st.partials = w.spart;
        st.pstride = partial_stride(c);
        return launch_stage(c, st);
    }
    laph_status clov(int prec, int parity, int inverse, Operand in, Operand out, int post, Operand y, double a,
                     double b) {
        CloverSpec cs;
        cs.prec = prec;
        cs.parity = parity;
        cs.inverse = inverse;
        cs.post = post;
        cs.in = in;
        cs.out = out;
        cs.y = y;
        cs.a = a;
        cs.b = b;
        cs.mass_idx = s.mass_idx;
        cs.n = n;
        return launch_clover(c, cs);
    }
    laph_status smooth(Operand r, Operand out);
    laph_status coarse_solve();
    laph_status vcycle(Operand r, Operand e);
    laph_status apply_d32(Operand in, Operand out);
    laph_status apply_d64(Operand in, Operand out);
    laph_status true_residual(int what, double tol);
    laph_status poll(std::vector<GcrState> &h) {
        h.resize(n);
        LAPH_HIP(hipMemcpyAsync(h.data(), w.gst, n * sizeof(GcrState), hipMemcpyDeviceToHost, c.stream));
        LAPH_HIP(hipStreamSynchronize(c.stream));
        return LAPH_OK;
    }
};

laph_status MgSolver::init_tiles() {
    const int cnt = ntiles * nr + ntiles + 1;
    hipLaunchKernelGGL(mg_tiles_kernel, dim3((cnt + 255) / 256), dim3(256), 0, c.stream, w.tiles, n, nr, ntiles,
                       s.mass_idx);
    return check_launch("mg_tiles_kernel");
}

// out ~ D^-1 r (FP32 full vectors): b^ from r, smooth_iters MR steps on M^ from
// zero, odd half by reconstruction.  Leaves the MR residual in sb (even half).
laph_status MgSolver::smooth(Operand r, Operand out) {
    const Operand re = half(r, 0, h32), ro = half(r, 1, h32);
    const Operand ai = half(w.sa, 1, h32), bh = half(w.sa, 0, h32);   // A_oo^-1 r_o, A_ee^-1 r_e
    const Operand rho = half(w.sb, 0, h32), tmp = half(w.sb, 1, h32);
    const Operand te = half(w.hq, 0, h32);
    const Operand oe = half(out, 0, h32), oo = half(out, 1, h32);
    LAPH_TRY(clov(LAPH_F32, 1, 1, ro, ai, 0, Operand{}, 0, 1));
    LAPH_TRY(clov(LAPH_F32, 0, 1, re, bh, 0, Operand{}, 0, 1));
    // rho = b^ = A_ee^-1 r_e + 1/2 A_ee^-1 H_eo A_oo^-1 r_o
    LAPH_TRY(stage(0, ai, rho, 1, 1, bh, 1.0, 0.5, 1, bh));
    hipLaunchKernelGGL(mg_zero_half_kernel, grid2(c.g.vh, n), dim3(kMB), 0, c.stream, c.g.vh, oe);
    LAPH_TRY(check_launch("mg_zero_half_kernel"));
    for (int it = 0; it < s.smooth_iters; ++it) {
        LAPH_TRY(stage(1, rho, tmp, 1, 0, Operand{}, 0, 1.0, 0, Operand{}));
        // t = rho - 1/4 A_ee^-1 H_eo tmp = M^ rho, with <t, rho> and |t|^2
        LAPH_TRY(stage(0, tmp, te, 1, 1, rho, 1.0, -0.25, 2, Operand{}));
        LAPH_TRY(sum_stage_partials(c, w.spart, partial_stride(c), stage_nsb(c, kFormLds), n, 3, w.dots));
        hipLaunchKernelGGL(mg_mr_update_kernel, grid2(c.g.vh, n), dim3(kMB), 0, c.stream, c.g.vh, (const double *)w.dots,
                           oe, rho, te);
        LAPH_TRY(check_launch("mg_mr_update_kernel"));
    }
    // e_o = A_oo^-1 r_o + 1/2 A_oo^-1 H_oe e_e
    LAPH_TRY(stage(1, oe, oo, 1, 1, ai, 1.0, 0.5, 1, ai));
    return LAPH_OK;
}

// out = D in on FP32 full vectors (hq as scratch)
laph_status MgSolver::apply_d32(Operand in, Operand out) {
    for (int p = 0; p < 2; ++p)
        LAPH_TRY(stage(p, half(in, 1 - p, h32), half(w.hq, p, h32), 0, 0, Operand{}, 0, -0.5, 0, Operand{}));
    for (int p = 0; p < 2; ++p)
        LAPH_TRY(clov(LAPH_F32, p, 0, half(in, p, h32), half(out, p, h32), 1, half(w.hq, p, h32), 1.0, 1.0));
    return LAPH_OK;
}

laph_status MgSolver::coarse_solve() {
    const size_t len = (size_t)s.geo.nc * s.geo.ncv;
    const dim3 g(cblk, n);
    auto upd = [&](int kind) {
        hipLaunchKernelGGL(mg_cupdate_kernel, g, dim3(kMB), 0, c.stream, (const CgState *)w.cst, kind, len, w.cx, w.cr,
                           w.crh, w.cp, w.cv, w.cs, w.ct, (const double2 *)w.cb);
        return check_launch("mg_cupdate_kernel");
    };
    auto dot = [&](const double2 *a0, const double2 *b0, const double2 *a1, const double2 *b1, int nq, int what) {
        hipLaunchKernelGGL(mg_cdot_kernel, g, dim3(kMB), 0, c.stream, a0, b0, a1, b1, nq, len, w.bpart);
        LAPH_TRY(check_launch("mg_cdot_kernel"));
        hipLaunchKernelGGL(mg_cscalar_kernel, dim3(n), dim3(kMB), 0, c.stream, w.cst, (const double *)w.bpart, cblk,
                           what, s.coarse_tol);
        return check_launch("mg_cscalar_kernel");
    };
    LAPH_TRY(upd(3));
    LAPH_TRY(dot(w.cb, w.cb, nullptr, nullptr, 1, kCgInit));
    for (int it = 0; it < s.coarse_iters; ++it) {
        LAPH_TRY(dot(w.crh, w.cr, nullptr, nullptr, 1, kCgRho));
        LAPH_TRY(upd(0));
        LAPH_TRY(coarse_apply_dev(c, w.cv, w.cp, n));
        LAPH_TRY(dot(w.crh, w.cv, nullptr, nullptr, 1, kCgAlpha));
        LAPH_TRY(upd(1));
        LAPH_TRY(coarse_apply_dev(c, w.ct, w.cs, n));
        LAPH_TRY(dot(w.ct, w.cs, w.ct, w.ct, 2, kCgOmega));
        LAPH_TRY(upd(2));
        LAPH_TRY(dot(w.cr, w.cr, nullptr, nullptr, 1, kCgRes));
    }
    return LAPH_OK;
}

// e ~ D^-1 r: pre-smoother, coarse correction of its residual, post-smoother
laph_status MgSolver::vcycle(Operand r, Operand e) {
    const MgDev m = mg_dev(s.geo);
    LAPH_TRY(smooth(r, e));
    // residual of the pre-smoothed e: (A_ee rho, 0)
    LAPH_TRY(clov(LAPH_F32, 0, 0, half(w.sb, 0, h32), half(w.res, 0, h32), 0, Operand{}, 0, 1.0));
    const int ng = (n + kMgRhsGroup - 1) / kMgRhsGroup;
    hipLaunchKernelGGL(mg_restrict32_kernel, dim3(s.geo.nc, ng), dim3(kMB), 0, c.stream, c.g, m,
                       (const char *)s.basis32, s.basis32_stride, h32, w.res, h32, 1, n, w.cb);
    LAPH_TRY(check_launch("mg_restrict32_kernel"));
    LAPH_TRY(coarse_solve());
    hipLaunchKernelGGL((mg_prolong32_kernel<false>), dim3((2 * c.g.vh + kMB - 1) / kMB, ng), dim3(kMB), 0, c.stream,
                       c.g, m, (const char *)s.basis32, s.basis32_stride, h32, (const double2 *)w.cx, w.q, h32, n);
    LAPH_TRY(check_launch("mg_prolong32_kernel"));
    hipLaunchKernelGGL(mg_add_kernel<F32>, grid2(2 * c.g.vh, n), dim3(kMB), 0, c.stream, c.g.vh, 2, h32, e, e, w.q);
    LAPH_TRY(check_launch("mg_add_kernel"));
    // res2 = res - D q: hq = 1/2 H q; hq += res (odd residual half is zero); res2 = hq - A q
    for (int p = 0; p < 2; ++p)
        LAPH_TRY(stage(p, half(w.q, 1 - p, h32), half(w.hq, p, h32), 0, 0, Operand{}, 0, 0.5, 0, Operand{}));
    hipLaunchKernelGGL(mg_add_kernel<F32>, grid2(c.g.vh, n), dim3(kMB), 0, c.stream, c.g.vh, 1, h32,
                       half(w.hq, 0, h32), half(w.hq, 0, h32), half(w.res, 0, h32));
    LAPH_TRY(check_launch("mg_add_kernel"));
    for (int p = 0; p < 2; ++p)
        LAPH_TRY(clov(LAPH_F32, p, 0, half(w.q, p, h32), half(w.res, p, h32), 1, half(w.hq, p, h32), 1.0, -1.0));
    LAPH_TRY(smooth(w.res, w.q));
    hipLaunchKernelGGL(mg_add_kernel<F32>, grid2(2 * c.g.vh, n), dim3(kMB), 0, c.stream, c.g.vh, 2, h32, e, e, w.q);
    return check_launch("mg_add_kernel");
}

// r = b - D x in FP64 (what 0: x = 0 start; 2: a reliable update), with the status update
laph_status MgSolver::apply_d64(Operand in, Operand out) {
    for (int p = 0; p < 2; ++p)
        LAPH_TRY(clov(LAPH_F64, p, 0, half(in, p, h64), half(out, p, h64), 0, Operand{}, 0, 1.0));
    for (int p = 0; p < 2; ++p) {
        // out_p = A_pp in_p - 1/2 H in_(1-p): the FP64 stage reads its xpay term from out
        StageSpec st;
        st.prec = LAPH_F64;
        st.form = kFormLds;
        st.site_major = 1;
        st.out_parity = p;
        st.post = 1;
        st.in = half(in, 1 - p, h64);
        st.out = half(out, p, h64);
        st.y = half(out, p, h64);
        st.a = 1.0;
        st.b = -0.5;
        st.tiles = tiles();   // the FP64 LDS stage takes tiles of 4, 8 or 16 RHS as well
        st.pstride = partial_stride(c);
        st.partials = w.spart;
        LAPH_TRY(launch_stage(c, st));
    }
    return LAPH_OK;
}

// r = b - D x in FP64 (what 0: x = 0 start; 2: a reliable update), with the status update
laph_status MgSolver::true_residual(int what, double tol) {
    LAPH_TRY(apply_d64(w.x, w.r));
    hipLaunchKernelGGL(mg_resid_kernel, dim3(nblk, n), dim3(kMB), 0, c.stream, c.g.vh, h64, w.b, w.r, w.bpart, what == 0 ? 1 : 0);
    LAPH_TRY(check_launch("mg_resid_kernel"));
    hipLaunchKernelGGL(mg_sum_kernel, dim3(n), dim3(kMB), 0, c.stream, (const double *)w.bpart, nblk, what == 0 ? 2 : 1,
                       2, w.sums);
    LAPH_TRY(check_launch("mg_sum_kernel"));
    hipLaunchKernelGGL(mg_gcr_status_kernel, dim3((n + 63) / 64), dim3(64), 0, c.stream, w.gst, (const double *)w.sums, 2,
                       n, what, tol);
    return check_launch("mg_gcr_status_kernel");
}

laph_status MgSolver::solve(double tol, std::vector<GcrState> &h) {
    LAPH_TRY(init_tiles());
    LAPH_HIP(hipMemsetAsync(w.x.base, 0, (size_t)n * w.x.stride, c.stream));
    LAPH_HIP(hipMemsetAsync(w.gst, 0, (size_t)n * sizeof(GcrState), c.stream));
    LAPH_TRY(true_residual(0, tol));
    const int m = s.restart;
    int it = 0;
    for (;;) {
        LAPH_TRY(poll(h));
        bool all = true;
        for (const auto &g : h) all = all && g.done;
        if (all || it >= s.maxiter) break;
        for (int k = 0; k < m && it < s.maxiter; ++k, ++it) {
            const Operand Zk = sub(w.Z, k), Wk = sub(w.W, k);
            hipLaunchKernelGGL((mg_convert_kernel<F64, F32>), grid2(2 * c.g.vh, n), dim3(kMB), 0, c.stream, c.g.vh,
                               h64, h32, w.r32, w.r);
            LAPH_TRY(check_launch("mg_convert_kernel"));
            LAPH_TRY(vcycle(w.r32, Zk));
            LAPH_TRY(apply_d32(Zk, Wk));
            if (k > 0) {
                hipLaunchKernelGGL(mg_gcr_multidot_kernel, dim3(nblk, n), dim3(kMB), 0, c.stream, c.g.vh, h32, w.W, m, k,
                                   w.bpart, (const GcrState *)w.gst);
                LAPH_TRY(check_launch("mg_gcr_multidot_kernel"));
                hipLaunchKernelGGL(mg_sum_kernel, dim3(n), dim3(kMB), 0, c.stream, (const double *)w.bpart, nblk, 2 * k,
                                   2 * kMgMaxRestart, w.sums);
                LAPH_TRY(check_launch("mg_sum_kernel"));
                hipLaunchKernelGGL(mg_gcr_orth_kernel, grid2(2 * c.g.vh, n), dim3(kMB), 0, c.stream, c.g.vh, h32, w.W,
                                   w.Z, m, k, (const double *)w.sums, (const GcrState *)w.gst);
                LAPH_TRY(check_launch("mg_gcr_orth_kernel"));
            }
            hipLaunchKernelGGL(mg_gcr_dot2_kernel, dim3(nblk, n), dim3(kMB), 0, c.stream, c.g.vh, h32, h64, w.W, m, k, w.r,
                               w.bpart, (const GcrState *)w.gst);
            LAPH_TRY(check_launch("mg_gcr_dot2_kernel"));
            hipLaunchKernelGGL(mg_sum_kernel, dim3(n), dim3(kMB), 0, c.stream, (const double *)w.bpart, nblk, 3, 3, w.sums);
            LAPH_TRY(check_launch("mg_sum_kernel"));
            hipLaunchKernelGGL(mg_gcr_scalar_kernel, dim3((n + 63) / 64), dim3(64), 0, c.stream, w.gst,
                               (const double *)w.sums, n);
            LAPH_TRY(check_launch("mg_gcr_scalar_kernel"));
            hipLaunchKernelGGL(mg_gcr_update_kernel, dim3(nblk, n), dim3(kMB), 0, c.stream, c.g.vh, h32, h64, w.W, w.Z, m,
                               k, w.x, w.r, w.bpart, (const GcrState *)w.gst);
            LAPH_TRY(check_launch("mg_gcr_update_kernel"));
            hipLaunchKernelGGL(mg_sum_kernel, dim3(n), dim3(kMB), 0, c.stream, (const double *)w.bpart, nblk, 1, 1, w.sums);
            LAPH_TRY(check_launch("mg_sum_kernel"));
            hipLaunchKernelGGL(mg_gcr_status_kernel, dim3((n + 63) / 64), dim3(64), 0, c.stream, w.gst,
                               (const double *)w.sums, 1, n, 1, tol);
            LAPH_TRY(check_launch("mg_gcr_status_kernel"));
            LAPH_TRY(poll(h));
            bool fr = true;
            for (const auto &g : h) fr = fr && g.frozen;
            if (fr) {
                ++it;
                break;
            }
        }
        // reliable update: the FP64 residual of x, and the restart of the directions
        LAPH_TRY(true_residual(2, tol));
    }
    return LAPH_OK;
}

// One building block of the cycle on n canonical fields (what 0: D in FP32; 1: the
// smoother; 2: the whole cycle) or n coarse vectors (3: the coarse BiCGStab).
laph_status MgSolver::component(int what, double *out, const double *in) {
    LAPH_TRY(init_tiles());
    if (what == 3) {
        const size_t bytes = (size_t)n * s.geo.nc * s.geo.ncv * sizeof(double2);
        LAPH_HIP(hipMemcpyAsync(w.cb, in, bytes, hipMemcpyDeviceToDevice, c.stream));
        LAPH_TRY(coarse_solve());
        LAPH_HIP(hipMemcpyAsync(out, w.cx, bytes, hipMemcpyDeviceToDevice, c.stream));
        return LAPH_OK;
    }
    LAPH_TRY(pack_spinor(c, w.b, in, LAPH_F64, n, -1, 0));
    if (what == 5 || what == 6) {
        // the normalised GCR directions Z (5) or W = D Z (6) after maxiter iterations, [k][n]
        std::vector<GcrState> h;
        LAPH_TRY(solve(1e-300, h));
        const size_t full = (size_t)2 * c.g.vh * 12 * 2;   // doubles per canonical field
        for (int k = 0; k < s.restart; ++k) {
            hipLaunchKernelGGL((mg_convert_kernel<F32, F64>), grid2(2 * c.g.vh, n), dim3(kMB), 0, c.stream, c.g.vh,
                               h32, h64, w.x, sub(what == 5 ? w.Z : w.W, k));
            LAPH_TRY(check_launch("mg_convert_kernel"));
            LAPH_TRY(unpack_spinor(c, out + (size_t)k * n * full, w.x, LAPH_F64, n, -1, 0));
        }
        return LAPH_OK;
    }
    if (what == 4) {
        LAPH_TRY(apply_d64(w.b, w.x));
        return unpack_spinor(c, out, w.x, LAPH_F64, n, -1, 0);
    }
    hipLaunchKernelGGL((mg_convert_kernel<F64, F32>), grid2(2 * c.g.vh, n), dim3(kMB), 0, c.stream, c.g.vh, h64, h32,
                       w.r32, w.b);
    LAPH_TRY(check_launch("mg_convert_kernel"));
    const Operand Z0 = sub(w.Z, 0);
    if (what == 0)
        LAPH_TRY(apply_d32(w.r32, Z0));
    else if (what == 1)
        LAPH_TRY(smooth(w.r32, Z0));
    else
        LAPH_TRY(vcycle(w.r32, Z0));
    hipLaunchKernelGGL((mg_convert_kernel<F32, F64>), grid2(2 * c.g.vh, n), dim3(kMB), 0, c.stream, c.g.vh, h32, h64,
                       w.x, Z0);
    LAPH_TRY(check_launch("mg_convert_kernel"));
    return unpack_spinor(c, out, w.x, LAPH_F64, n, -1, 0);
}

}  // namespace

size_t mg_solve_workspace_bytes(const Ctx &c, int nrhs, int restart) {
    return mg_layout(c, nrhs, restart, nullptr, nullptr);
}

laph_status mg_component(Ctx &c, const MgState &run, int what, double *out, const double *in, int n, char *work,
                         size_t work_bytes) {
    LAPH_TRY(need_mg(c));
    if (what < 0 || what > 6) return set_error(LAPH_ERR_INVALID, "multigrid component: what must be 0..6");
    if (work_bytes < mg_layout(c, n, run.restart, nullptr, nullptr))
        return set_error(LAPH_ERR_WORKSPACE, "multigrid workspace too small");
    MgWs w;
    mg_layout(c, n, run.restart, work, &w);
    MgSolver solver(c, run, n, w);
    LAPH_TRY(solver.component(what, out, in));
    LAPH_HIP(hipStreamSynchronize(c.stream));
    return LAPH_OK;
}

laph_status mg_solve(Ctx &c, const MgState &run, double *X, const double *B, int nrhs, double tol,
                     laph_rhs_stats *stats, char *work, size_t work_bytes) {
    LAPH_TRY(need_mg(c));
    if (work_bytes < mg_layout(c, nrhs, run.restart, nullptr, nullptr))
        return set_error(LAPH_ERR_WORKSPACE, "multigrid solve workspace too small");
    MgWs w;
    mg_layout(c, nrhs, run.restart, work, &w);
    LAPH_TRY(pack_spinor(c, w.b, B, LAPH_F64, nrhs, -1, 0));
    MgSolver solver(c, run, nrhs, w);
    LAPH_HIP(hipEventRecord(c.ev[0], c.stream));
    std::vector<GcrState> h;
    LAPH_TRY(solver.solve(tol, h));
    LAPH_TRY(unpack_spinor(c, X, w.x, LAPH_F64, nrhs, -1, 0));
    LAPH_HIP(hipEventRecord(c.ev[1], c.stream));
    LAPH_HIP(hipEventSynchronize(c.ev[1]));
    float ms = 0;
    LAPH_HIP(hipEventElapsedTime(&ms, c.ev[0], c.ev[1]));
    c.last_ms[0] = c.last_ms[1] = ms;
    int worst = LAPH_OK;
    for (int r = 0; r < nrhs; ++r) {
        const double tr = std::sqrt(h[r].true_res2);
        int status = h[r].done && tr <= tol ? LAPH_RHS_CONVERGED : LAPH_RHS_NOCONV;
        if (!std::isfinite(tr)) status = LAPH_RHS_NONFINITE;
        if (stats) {
            stats[r].status = status;
            stats[r].iters = h[r].iters;
            stats[r].updates = h[r].restarts;
            stats[r].restarts = 0;
            stats[r].true_res = tr;
        }
        if (status == LAPH_RHS_NONFINITE)
            worst = LAPH_ERR_NONFINITE;
        else if (status != LAPH_RHS_CONVERGED && worst == LAPH_OK)
            worst = LAPH_ERR_NOCONV;
    }
    if (worst != LAPH_OK) return set_error((laph_status)worst, "multigrid solve: some right-hand sides did not converge (see stats)");
    return LAPH_OK;
}

}  // namespace laph
