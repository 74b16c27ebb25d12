// LapH eigenvectors on the GPU: the lowest nev eigenpairs of the gauge-covariant
// 3-D Laplacian -Delta on every timeslice (the paper's Sec. "LapH" / "QUDA": the
// LapH subspace is spanned by the lowest eigenvectors of the gauge-covariant
// Laplacian of each time slice; computing them on the GPU is the paper's new step).
//
// (-Delta f)(x) = sum_{k=x,y,z} [2 f(x) - U_k(x) f(x+k) - U_k(x-k)^dagger f(x-k)],
// periodic, no boundary phase; spectrum inside [0, 12] for unitary links.
//
// Method: Chebyshev-filtered subspace iteration, all timeslices at once.  Per
// iteration and timeslice, a block of m = nev + guard vectors is filtered by the
// degree-d Chebyshev polynomial that damps [lambda_cut, 12] (lambda_cut = the
// largest Ritz value of the block; d as large as allowed while the growth of the
// lowest Ritz direction over the cut stays below ~1e6), made orthonormal by two
// Cholesky passes (Gram matrix C = R^dagger R, Y <- Y R^{-1}; the first pass shifted by
// 1e-15 of the largest Gram diagonal entry; a timeslice whose factorisation breaks
// down takes Y <- Y Q Lambda^{-1/2} from the Gram matrix's eigendecomposition
// instead), and rotated to Ritz vectors by a Rayleigh-Ritz step; it stops when every one of the nev lowest Ritz
// pairs has ||(-Delta) y - lambda y|| <= tol.  Every vector operation runs here:
// the stencil (links staged in LDS once per block of sites for a group of vectors,
// FP64), the Gram matrices and the block rotations (FP64 matrix cores), the small
// Hermitian eigenproblems and Cholesky factors (one workgroup per timeslice, matrix
// in LDS) and the residual norms.
//
// Layout of a block: [t][j][a][z][y][x] complex double (colour planes, so the
// stencil's loads are contiguous across the lanes of a wave), vectors of one
// timeslice contiguous; the result is written in the canonical V layout
// [t][l][z][y][x][a].
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <initializer_list>
#include <vector>

#include "laph_solver.h"

namespace laph {

namespace {

constexpr int kLB = 256;          // threads per block of the vector kernels
constexpr int kEigMaxM = 96;      // largest block (Jacobi matrix in LDS)
constexpr int kJB = 1024;         // threads of the Jacobi workgroup
constexpr int kGKC = 16;          // Gram K chunk
constexpr int kLmax = 12;         // upper bound of the spectrum
constexpr int kDefaultDegree = 96; // Chebyshev degree cap when the caller passes <= 1 (the growth
                                   // bound below is what limits it: about 65 at 32^3)

// ---- stencil: out = ca[t] (-Delta) in + cb[t] in + cc[t] z ------------------------
struct LapArgs {
    Geom g;
    GaugePtrs gp;
    const double2 *in, *z;
    double2 *out;
    int m;                  // vectors per timeslice in the block
    int nvec;               // vectors to process (first nvec of each timeslice)
    const double *coef;     // [lt][3] (ca, cb, cc); null: (1, 0, 0)
};

__device__ __forceinline__ void site3(const Geom &g, int s, int &x, int &y, int &z) {
    x = s % g.lx;
    const int r = s / g.lx;
    y = r % g.ly;
    z = r / g.ly;
}

// A workgroup owns kLapSites sites of one timeslice: its threads first stage the 6
// links of those sites in LDS (backward ones already as U^dagger) with the
// neighbour indices, then each wave runs two vectors at a time (lanes 0-31 and
// 32-63), so every link is read from HBM once for all vectors of the block.
constexpr int kLapSites = 32;
// vectors per group (grid dimension, outermost): groups re-stage the links, all-vector
// blocks lose the L2 reuse of their neighbour rows.  At 32^3 x 64 with 96 vectors and
// rows in memory order, 32 measured best (4.03 s for an earlier eigensolver, against
// 4.24 s with one group of all vectors, 4.19 s with 16 and 4.46 s with 8); with the
// (y, z) row tiles below, 48 (2.81 s, against 2.88 s with 32 and 2.95 s with 96)
#ifndef LAPH_LAP_VG
#define LAPH_LAP_VG 48
#endif
// rows of a timeslice (one row = kLapSites sites) visited in T x T tiles of (y, z)
// when the x extent is one row (0: memory order), so the blocks in flight hold more of
// each other's y and z neighbours: at 32^3 x 64 with 96 vectors the eigensolver took
// 3.00 s in memory order, 3.00 s with tiles of 2, 2.88 s with 4, 2.85-2.88 s with 8
// and 2.87 s with 16
#ifndef LAPH_LAP_TILE
#define LAPH_LAP_TILE 4
#endif

// element (site, colour) of a vector: colour planes (Planar) or the canonical
// site-major order
template <bool HasZ, bool Planar>
__global__ __launch_bounds__(kLB) void lap_kernel(LapArgs A) {
    __shared__ double lnk[6][18][kLapSites];
    __shared__ int nbr[6][kLapSites];
    const Geom &g = A.g;
    const int vs = g.lx * g.ly * g.lz;
    // XCD-aware order: consecutive workgroup ids go round-robin over the 8 XCDs, so id
    // b is remapped to give each XCD a contiguous range of (timeslice, row) blocks; the
    // y and z neighbour rows of a block then run on the same XCD, close in time, and
    // their vectors are shared in its L2
    const int nrow = (vs + kLapSites - 1) / kLapSites;
    const int nblk = gridDim.x;
    int bid = blockIdx.x;
    if (nblk % 8 == 0) bid = (bid % 8) * (nblk / 8) + bid / 8;
    // vector groups outermost: the blocks in flight work on the same few vectors, so
    // the y and z neighbour rows a block reads were loaded by its neighbours moments ago
    const int grp = bid / (nrow * g.lt);
    bid -= grp * nrow * g.lt;
    const int t = bid / nrow;
    int row = bid - t * nrow;
    if (LAPH_LAP_TILE > 0 && g.lx == kLapSites && g.ly % LAPH_LAP_TILE == 0 && g.lz % LAPH_LAP_TILE == 0) {
        constexpr int T = LAPH_LAP_TILE > 0 ? LAPH_LAP_TILE : 1;
        const int in_tile = row % (T * T), tile = row / (T * T);
        const int nyt = g.ly / T;
        row = ((tile / nyt) * T + in_tile / T) * g.ly + (tile % nyt) * T + in_tile % T;
    }
    const int s0 = row * kLapSites;
    const int j_lo = grp * LAPH_LAP_VG, j_hi = min(A.nvec, j_lo + LAPH_LAP_VG);
    // ---- phase 1: links and neighbours (thread -> (hop, site))
    for (int q = threadIdx.x; q < 6 * kLapSites; q += kLB) {
        const int hop = q / kLapSites, site = q - hop * kLapSites;
        const int s = s0 + site;
        const int k = hop >> 1, fb = hop & 1;
        cplx<double> L[9];
        int sn = 0;
        if (s < vs) {
            int x, y, z;
            site3(g, s, x, y, z);
            int nx = x, ny = y, nz = z;
            if (k == 0) nx = fb == 0 ? (x + 1 == g.lx ? 0 : x + 1) : (x == 0 ? g.lx - 1 : x - 1);
            if (k == 1) ny = fb == 0 ? (y + 1 == g.ly ? 0 : y + 1) : (y == 0 ? g.ly - 1 : y - 1);
            if (k == 2) nz = fb == 0 ? (z + 1 == g.lz ? 0 : z + 1) : (z == 0 ? g.lz - 1 : z - 1);
            sn = nx + g.lx * (ny + g.ly * nz);
            // forward: U_k(x); backward: U_k(x - k)^dagger
            const int lx_ = fb == 0 ? x : nx, ly_ = fb == 0 ? y : ny, lz_ = fb == 0 ? z : nz;
            GaugeIO<F64>::load(A.gp, (lx_ + ly_ + lz_ + t) & 1, k, g.vh, cb_index(g, lx_, ly_, lz_, t), L);
        } else {
#pragma unroll
            for (int e = 0; e < 9; ++e) L[e] = {0.0, 0.0};
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const cplx<double> e = fb == 0 ? L[a * 3 + b] : conj(L[b * 3 + a]);
                lnk[hop][2 * (a * 3 + b)][site] = e.re;
                lnk[hop][2 * (a * 3 + b) + 1][site] = e.im;
            }
        nbr[hop][site] = sn;
    }
    __syncthreads();
    // ---- phase 2: vectors, two per wave per round
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int site = lane & (kLapSites - 1), vsub = lane >> 5;
    const int s = s0 + site;
    if (s >= vs) return;
    double ca = 1.0, cb = 0.0, cc = 0.0;
    if (A.coef) {
        ca = A.coef[3 * t];
        cb = A.coef[3 * t + 1];
        cc = A.coef[3 * t + 2];
    }
    const size_t tb = (size_t)t * A.m;
    const int ss = Planar ? 1 : 3, sa = Planar ? vs : 1;
    int nb[6];
#pragma unroll
    for (int hop = 0; hop < 6; ++hop) nb[hop] = nbr[hop][site] * ss;
#pragma unroll 1
    for (int j = j_lo + 2 * wave + vsub; j < j_hi; j += 2 * (kLB / 64)) {
        const size_t vb = (tb + j) * vs * 3;
        const double2 *__restrict__ vin = A.in + vb;
        // every load of this vector first (six neighbours, the site itself, z), so a
        // wave keeps up to 24 loads in flight; then the products with the staged links
        double2 fn[6][3], fc[3], fz[3];
#pragma unroll
        for (int hop = 0; hop < 6; ++hop)
#pragma unroll
            for (int a = 0; a < 3; ++a) fn[hop][a] = vin[nb[hop] + a * sa];
#pragma unroll
        for (int a = 0; a < 3; ++a) fc[a] = vin[ss * s + a * sa];
        if (HasZ) {
#pragma unroll
            for (int a = 0; a < 3; ++a) fz[a] = A.z[vb + ss * s + a * sa];
        }
        // the links are re-read from LDS per vector (an opaque index keeps the compiler
        // from holding all 108 of them in registers across the loop)
        int ls = site;
        asm volatile("" : "+v"(ls));
        cplx<double> acc[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
        for (int hop = 0; hop < 6; ++hop)
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const cplx<double> l = {lnk[hop][2 * (a * 3 + b)][ls], lnk[hop][2 * (a * 3 + b) + 1][ls]};
                    cmac(acc[a], l, cplx<double>{fn[hop][b].x, fn[hop][b].y});
                }
        double2 *__restrict__ vout = A.out + vb;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // (-Delta f) = 6 f - hops
            double re = ca * (6.0 * fc[a].x - acc[a].re) + cb * fc[a].x;
            double im = ca * (6.0 * fc[a].y - acc[a].im) + cb * fc[a].y;
            if (HasZ) {
                re += cc * fz[a].x;
                im += cc * fz[a].y;
            }
            vout[ss * s + a * sa] = make_double2(re, im);
        }
    }
}

// ---- Gram matrices C[t][i][j] = sum_e conj(P[t][i][e]) R[t][j][e] ---------------------
using d4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;

struct GramArgs {
    const double2 *P, *R;   // blocks [lt][m][ne]
    int m, ne, lt;
    int ntile;              // tiles per dimension
    int nsplit, nchunk;
    double2 *scratch;       // [split][lt][m][m]
};

// One workgroup per (timeslice, K slice) computes the m x m block (m <= 96: 6 x 6
// blocks of 16), so no tile padding is computed at m = 96 (tiles of 64 did 1.78x the
// work).  Both uses of C here are Hermitian (a Gram matrix Y^dagger Y, and
// H = Y^dagger (-Delta) Y), so only the 21 blocks on and above the diagonal are
// computed, at most 6 per wave (rows 0 | 1 | 2 and 5 | 3 and 4), and the second pass
// mirrors them.
__device__ __forceinline__ void gram_slot(int wave, int s, int &a, int &b) {
    if (wave == 0) { a = 0; b = s; }
    else if (wave == 1) { a = 1; b = 1 + s; }
    else if (wave == 2) { a = s < 4 ? 2 : 5; b = s < 4 ? 2 + s : 5; }
    else { a = s < 3 ? 3 : 4; b = s < 3 ? 3 + s : s + 1; }
}

__global__ __launch_bounds__(256) void gram_kernel(GramArgs A) {
    __shared__ double Pr[kEigMaxM][kGKC + 1], Pi[kEigMaxM][kGKC + 1], Rr[kEigMaxM][kGKC + 1], Ri[kEigMaxM][kGKC + 1];
    const int split = blockIdx.x % A.nsplit;
    const int t = blockIdx.x / A.nsplit;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nslot = wave == 0 ? 6 : 5;   // wave-uniform
    int sa[6], sb[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) gram_slot(wave, s, sa[s], sb[s]);
    d4 cre[6], cim[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        cre[s] = d4{0, 0, 0, 0};
        cim[s] = d4{0, 0, 0, 0};
    }
    const int c0 = (int)((long)A.nchunk * split / A.nsplit), c1 = (int)((long)A.nchunk * (split + 1) / A.nsplit);
    const double2 *P = A.P + (size_t)t * A.m * A.ne, *R = A.R + (size_t)t * A.m * A.ne;
    for (int ch = c0; ch < c1; ++ch) {
        // rows of P and R (zero past m), K = this chunk's 16 elements (zero past ne)
        for (int q = tid; q < kEigMaxM * kGKC; q += 256) {
            const int r = q / kGKC, kk = q - r * kGKC;
            const int e = ch * kGKC + kk;
            double2 pv = make_double2(0, 0), rv = make_double2(0, 0);
            if (e < A.ne && r < A.m) {
                pv = P[(size_t)r * A.ne + e];
                rv = R[(size_t)r * A.ne + e];
            }
            Pr[r][kk] = pv.x;
            Pi[r][kk] = pv.y;
            Rr[r][kk] = rv.x;
            Ri[r][kk] = rv.y;
        }
        __syncthreads();
#pragma unroll
        for (int k4 = 0; k4 < kGKC; k4 += 4) {
            const int kk = k4 + (lane >> 4);
            // conj(P) R = (Pr Rr + Pi Ri) + i (Pr Ri - Pi Rr)
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                if (s >= nslot) break;
                const int row = 16 * sa[s] + (lane & 15), col = 16 * sb[s] + (lane & 15);
                const double ar = Pr[row][kk], ai = Pi[row][kk], br = Rr[col][kk], bi = Ri[col][kk];
                cre[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, cre[s], 0, 0, 0);
                cim[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, cim[s], 0, 0, 0);
                cre[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, cre[s], 0, 0, 0);
                cim[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, br, cim[s], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // the 16x16x4 FP64 MFMA leaves C[row][col] in lane col + 16 (row % 4), register row / 4
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        if (s >= nslot) break;
        const int j = 16 * sb[s] + (lane & 15);
        if (j >= A.m) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * sa[s] + (lane >> 4) + 4 * r;
            if (i >= A.m) continue;
            A.scratch[(((size_t)split * A.lt + t) * A.m + i) * A.m + j] = make_double2(cre[s][r], cim[s][r]);
        }
    }
}

__global__ void gram_reduce_kernel(GramArgs A, double2 *C) {
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    const long total = (long)A.lt * A.m * A.m;
    if (idx >= total) return;
    // entries of blocks below the diagonal are the conjugates of their mirror images
    const long mm = (long)A.m * A.m, t = idx / mm;
    const int i = (int)((idx - t * mm) / A.m), j = (int)(idx - t * mm - (long)i * A.m);
    const bool mirror = i / 16 > j / 16;
    const long src = mirror ? t * mm + (long)j * A.m + i : idx;
    double2 s = make_double2(0, 0);
    for (int sp = 0; sp < A.nsplit; ++sp) {
        const double2 v = A.scratch[(size_t)sp * total + src];
        s.x += v.x;
        s.y += v.y;
    }
    C[idx] = mirror ? make_double2(s.x, -s.y) : s;
}

// ---- Hermitian eigensolver: cyclic Jacobi, round-robin parallel ordering ---------------
// One workgroup per timeslice.  C[t] (m x m, made Hermitian) -> eigenvalues w[t][m]
// ascending and Z[t][k][j]: mode 0 the eigenvector matrix, mode 1 Q Lambda^{-1/2}
// (columns of the Gram matrix's eigenvectors scaled; shift added to the eigenvalues).
struct JacArgs {
    const double2 *C;     // [lt][m][m]
    double2 *Q;           // [lt][m][m] work (eigenvectors, columns)
    double2 *Z;           // [lt][m][m] output
    double *w;            // [lt][m] output
    int m;
    int mode;
    double shift_rel;     // mode 1: shift = shift_rel * largest eigenvalue
    int max_sweeps;
    int *flag;            // [lt]: Cholesky writes 1 where it broke down; Jacobi, given
                          // the array, works only on those timeslices
    double tiny;          // Cholesky: smallest pivot accepted, relative to the largest diagonal
};

__global__ __launch_bounds__(kJB) void jacobi_kernel(JacArgs A) {
    __shared__ double hr[kEigMaxM * kEigMaxM], hi[kEigMaxM * kEigMaxM];
    __shared__ double rc[kEigMaxM / 2], rs[kEigMaxM / 2], rer[kEigMaxM / 2], rei[kEigMaxM / 2];
    __shared__ int rp[kEigMaxM / 2], rq[kEigMaxM / 2];
    __shared__ double red[kJB / 64][2];
    __shared__ int order[kEigMaxM];
    const int m = A.m, t = blockIdx.x, tid = threadIdx.x;
    if (A.flag && A.flag[t] == 0) return;
    const double2 *C = A.C + (size_t)t * m * m;
    double2 *Q = A.Q + (size_t)t * m * m;
    for (int e = tid; e < m * m; e += kJB) {
        const int i = e / m, j = e - i * m;
        const double2 a = C[i * m + j], b = C[j * m + i];
        hr[e] = 0.5 * (a.x + b.x);   // (C + C^dagger) / 2
        hi[e] = 0.5 * (a.y - b.y);
        Q[e] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    const int half = m / 2;
    for (int sweep = 0; sweep < A.max_sweeps; ++sweep) {
        // off-diagonal and total Frobenius norms (block reduction, fixed order)
        double off = 0, tot = 0;
        for (int e = tid; e < m * m; e += kJB) {
            const double v = hr[e] * hr[e] + hi[e] * hi[e];
            tot += v;
            if (e / m != e % m) off += v;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            off += __shfl_xor(off, o, 64);
            tot += __shfl_xor(tot, o, 64);
        }
        if ((tid & 63) == 0) {
            red[tid >> 6][0] = off;
            red[tid >> 6][1] = tot;
        }
        __syncthreads();
        off = tot = 0;
        for (int wv = 0; wv < kJB / 64; ++wv) {
            off += red[wv][0];
            tot += red[wv][1];
        }
        __syncthreads();
        if (!(off > 1e-30 * tot) || tot == 0.0) break;   // uniform over the block
        for (int r = 0; r < m - 1; ++r) {
            // pairs of this round (circle method: player 0 fixed, the others rotate)
            if (tid < half) {
                auto player = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + r) % (m - 1); };
                int p = player(tid), q = player(m - 1 - tid);
                if (p > q) {
                    const int tmp = p;
                    p = q;
                    q = tmp;
                }
                const double a = hr[p * m + p], d = hr[q * m + q];
                const double br = hr[p * m + q], bi = hi[p * m + q];
                const double ab = sqrt(br * br + bi * bi);
                double c = 1.0, s = 0.0, er = 1.0, ei = 0.0;
                if (ab > 1e-300) {
                    er = br / ab;
                    ei = bi / ab;
                    const double tau = (d - a) / (2.0 * ab);
                    const double tt = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + tt * tt);
                    s = tt * c;
                }
                rp[tid] = p;
                rq[tid] = q;
                rc[tid] = c;
                rs[tid] = s;
                rer[tid] = er;
                rei[tid] = ei;
            }
            __syncthreads();
            // J = [[c, s], [-s conj(e), c conj(e)]] on (p, q).  Rows: H <- J^dagger H
            for (int e = tid; e < half * m; e += kJB) {
                const int k = e / m, col = e - k * m;
                const int p = rp[k], q = rq[k];
                const double c = rc[k], s = rs[k], er = rer[k], ei = rei[k];
                const double pr = hr[p * m + col], pi = hi[p * m + col];
                const double qr = hr[q * m + col], qi = hi[q * m + col];
                // conj(j00) = c, conj(j10) = -s e, conj(j01) = s, conj(j11) = c e
                hr[p * m + col] = c * pr - s * (er * qr - ei * qi);
                hi[p * m + col] = c * pi - s * (er * qi + ei * qr);
                hr[q * m + col] = s * pr + c * (er * qr - ei * qi);
                hi[q * m + col] = s * pi + c * (er * qi + ei * qr);
            }
            __syncthreads();
            // columns: H <- H J, Q <- Q J
            for (int e = tid; e < half * m; e += kJB) {
                const int k = e / m, row = e - k * m;
                const int p = rp[k], q = rq[k];
                const double c = rc[k], s = rs[k], er = rer[k], ei = rei[k];
                // j00 = c, j10 = -s conj(e), j01 = s, j11 = c conj(e)
                {
                    const double pr = hr[row * m + p], pi = hi[row * m + p];
                    const double qr = hr[row * m + q], qi = hi[row * m + q];
                    hr[row * m + p] = c * pr - s * (qr * er + qi * ei);
                    hi[row * m + p] = c * pi - s * (qi * er - qr * ei);
                    hr[row * m + q] = s * pr + c * (qr * er + qi * ei);
                    hi[row * m + q] = s * pi + c * (qi * er - qr * ei);
                }
                {
                    const double2 qp = Q[row * m + p], qq = Q[row * m + q];
                    Q[row * m + p] = make_double2(c * qp.x - s * (qq.x * er + qq.y * ei),
                                                  c * qp.y - s * (qq.y * er - qq.x * ei));
                    Q[row * m + q] = make_double2(s * qp.x + c * (qq.x * er + qq.y * ei),
                                                  s * qp.y + c * (qq.y * er - qq.x * ei));
                }
            }
            __syncthreads();
        }
    }
    // ascending order (ties by index), eigenvalues and the output matrix
    for (int i = tid; i < m; i += kJB) order[i] = i;
    __syncthreads();
    for (int i = tid; i < m; i += kJB) {
        const double wi = hr[i * m + i];
        int rank = 0;
        for (int j = 0; j < m; ++j) {
            const double wj = hr[j * m + j];
            rank += (wj < wi) || (wj == wi && j < i);
        }
        order[rank] = i;
    }
    __syncthreads();
    double wmax = hr[0];
    for (int i = 1; i < m; ++i) wmax = fmax(wmax, hr[i * m + i]);
    const double shift = A.mode == 1 ? A.shift_rel * wmax : 0.0;
    for (int e = tid; e < m * m; e += kJB) {
        const int k = e / m, j = e - k * m;
        const int src = min(max(order[j], 0), m - 1);
        double2 v = Q[k * m + src];
        if (A.mode == 1) {
            const double lam = fmax(hr[src * m + src], 0.0) + shift;
            const double sc = lam > 0 ? 1.0 / sqrt(lam) : 0.0;
            v.x *= sc;
            v.y *= sc;
        }
        A.Z[(size_t)t * m * m + e] = v;
    }
    for (int j = tid; j < m; j += kJB) {
        const int src = min(max(order[j], 0), m - 1);
        A.w[(size_t)t * m + j] = hr[src * m + src];
    }
}

// ---- orthonormalising factor: Z[t] = R^{-1} for C[t] + shift = R^dagger R ---------------
// One workgroup per timeslice, the Gram matrix in LDS: a right-looking Cholesky
// factorisation C + s I = L L^dagger (s = shift_rel times the largest diagonal entry),
// then X = L^{-1} by forward substitution (one column per thread) and Z = X^dagger, so
// the columns of Y Z are orthonormal: (Y Z)^dagger (Y Z) = X C X^dagger = I.  A pivot
// below `tiny` (1e-12) of the largest diagonal entry (a block too close to rank
// deficiency for two Cholesky passes to reach FP64 orthonormality) flags the
// timeslice, which the eigendecomposition then handles instead.
constexpr double kCholTiny = 1e-12;

__global__ __launch_bounds__(256) void chol_kernel(JacArgs A) {
    __shared__ double gr[kEigMaxM * kEigMaxM], gi[kEigMaxM * kEigMaxM];
    __shared__ double dmax;
    const int m = A.m, t = blockIdx.x, tid = threadIdx.x;
    const double2 *C = A.C + (size_t)t * m * m;
    for (int e = tid; e < m * m; e += 256) {
        const int i = e / m, j = e - i * m;
        const double2 a = C[i * m + j], b = C[j * m + i];
        gr[e] = 0.5 * (a.x + b.x);   // (C + C^dagger) / 2
        gi[e] = 0.5 * (a.y - b.y);
    }
    __syncthreads();
    if (tid == 0) {
        double d = 0.0;
        for (int i = 0; i < m; ++i) d = fmax(d, gr[i * m + i]);
        dmax = d;
    }
    __syncthreads();
    for (int i = tid; i < m; i += 256) gr[i * m + i] += A.shift_rel * dmax;
    __syncthreads();
    bool ok = true;
    for (int k = 0; k < m; ++k) {
        const double p = gr[k * m + k];
        ok = ok && p >= A.tiny * dmax;   // false for NaN too
        const double d = sqrt(fmax(p, 1e-300));
        __syncthreads();
        // column k below the diagonal: L[i][k] = G[i][k] / d
        for (int i = k + 1 + tid; i < m; i += 256) {
            gr[i * m + k] /= d;
            gi[i * m + k] /= d;
        }
        if (tid == 0) {
            gr[k * m + k] = d;
            gi[k * m + k] = 0.0;
        }
        __syncthreads();
        // trailing lower triangle: G[i][j] -= L[i][k] conj(L[j][k]), k < j <= i
        const int n = m - k - 1;
        for (int q = tid; q < n * n; q += 256) {
            const int i = k + 1 + q / n, j = k + 1 + q % n;
            if (j > i) continue;
            const double lr = gr[i * m + k], li = gi[i * m + k], rr = gr[j * m + k], ri = gi[j * m + k];
            gr[i * m + j] -= lr * rr + li * ri;
            gi[i * m + j] -= li * rr - lr * ri;
        }
        __syncthreads();
    }
    if (tid == 0) A.flag[t] = ok ? 0 : 1;
    // X = L^{-1}: column c solves L x = e_c (x[i] = 0 for i < c); Z[c][i] = conj(X[i][c]),
    // so row c of Z holds conj(x) and the substitution reads its own earlier entries back
    double2 *Z = A.Z + (size_t)t * m * m;
    for (int c = tid; c < m; c += 256) {
        double2 *zc = Z + (size_t)c * m;
        for (int i = 0; i < c; ++i) zc[i] = make_double2(0.0, 0.0);
        for (int i = c; i < m; ++i) {
            double sr = i == c ? 1.0 : 0.0, si = 0.0;
            for (int j = c; j < i; ++j) {
                const double lr = gr[i * m + j], li = gi[i * m + j];
                const double xr = zc[j].x, xi = -zc[j].y;
                sr -= lr * xr - li * xi;
                si -= lr * xi + li * xr;
            }
            const double dd = gr[i * m + i];
            zc[i] = make_double2(sr / dd, -si / dd);
        }
    }
}

// ---- block rotation: out[t][j] = sum_k in[t][k] Z[t][k][j] (first nout columns) ---------
struct RotArgs {
    const double2 *in;
    double2 *out;
    const double2 *Z;       // [lt][m][m]
    int m, ne, nout, mout;  // out block has mout vectors per timeslice
    const int *tri;         // [lt] or null: where tri[t] == 0, Z[t][k][j] = 0 for k > j
};

// Computed on the FP64 matrix cores as
// out^T[j][e] = sum_k Z^T[j][k] in[k][e] per timeslice: A = Z^T (rows j, staged in LDS
// 16 k at a time and shared by the four waves), B = the input block (16 consecutive e
// per k row: 256-byte loads), complex as four real products per 16 x 16 block.  A wave
// owns 32 e (two column blocks) and every j (up to six row blocks), so a lane's results
// for one j are 16 consecutive e: the stores are 256-byte segments too.  An upper
// triangular Z (a Cholesky factor's inverse) skips the row blocks wholly below the
// diagonal: 21 of the 36 block products at m = 96.
constexpr int kRE = 32;                 // e per wave
constexpr int kRK = 16;                 // k per staged chunk
constexpr int kRJB = kEigMaxM / 16;     // row blocks (j)

__global__ __launch_bounds__(256) void rotate_mfma_kernel(RotArgs A) {
    __shared__ double zr[kRK][kEigMaxM + 1], zi[kRK][kEigMaxM + 1];
    const int t = blockIdx.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e0 = (blockIdx.x * 4 + wave) * kRE;
    const int njb = (A.nout + 15) / 16;
    const bool upper = A.tri && A.tri[t] == 0;
    d4 cr[kRJB][2], ci[kRJB][2];
#pragma unroll
    for (int jb = 0; jb < kRJB; ++jb)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            cr[jb][c] = d4{0, 0, 0, 0};
            ci[jb][c] = d4{0, 0, 0, 0};
        }
    const double2 *in = A.in + (size_t)t * A.m * A.ne;
    const double2 *Zt = A.Z + (size_t)t * A.m * A.m;
    for (int k0 = 0; k0 < A.m; k0 += kRK) {
        // Z rows k0 .. k0 + 15, the first nout columns (zero elsewhere)
        for (int q = threadIdx.x; q < kRK * kEigMaxM; q += 256) {
            const int kk = q / kEigMaxM, j = q - kk * kEigMaxM;
            double2 v = make_double2(0.0, 0.0);
            if (k0 + kk < A.m && j < A.nout) v = Zt[(size_t)(k0 + kk) * A.m + j];
            zr[kk][j] = v.x;
            zi[kk][j] = v.y;
        }
        __syncthreads();
#pragma unroll
        for (int k4 = 0; k4 < kRK; k4 += 4) {
            const int kk = k4 + (lane >> 4), k = k0 + kk;
            double br[2], bi[2];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int e = e0 + 16 * c + (lane & 15);
                double2 v = make_double2(0.0, 0.0);
                if (k < A.m && e < A.ne) v = in[(size_t)k * A.ne + e];
                br[c] = v.x;
                bi[c] = v.y;
            }
#pragma unroll
            for (int jb = 0; jb < kRJB; ++jb) {
                if (jb >= njb) break;   // wave-uniform
                if (upper && 16 * jb + 15 < k0) continue;
                const int j = 16 * jb + (lane & 15);
                const double ar = zr[kk][j], ai = zi[kk][j], nai = -ai;
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    cr[jb][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br[c], cr[jb][c], 0, 0, 0);
                    cr[jb][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai, bi[c], cr[jb][c], 0, 0, 0);
                    ci[jb][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi[c], ci[jb][c], 0, 0, 0);
                    ci[jb][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br[c], ci[jb][c], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    // lane holds rows (lane >> 4) + 4 i of column lane & 15 of each 16 x 16 block
#pragma unroll
    for (int jb = 0; jb < kRJB; ++jb) {
        if (jb >= njb) break;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int e = e0 + 16 * c + (lane & 15);
            if (e >= A.ne) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int j = 16 * jb + (lane >> 4) + 4 * i;
                if (j < A.nout) A.out[((size_t)t * A.mout + j) * A.ne + e] = make_double2(cr[jb][c][i], ci[jb][c][i]);
            }
        }
    }
}

// ---- residual norms: r2[t][j] = || W[t][j] - w[t][j] Y[t][j] ||^2 -----------------------
__global__ __launch_bounds__(kLB) void residual_kernel(const double2 *Y, const double2 *W, const double *w, double *r2,
                                                       int m, int ne, int nvec) {
    __shared__ double red[kLB / 64];
    const int j = blockIdx.x, t = blockIdx.y;
    if (j >= nvec) return;
    const double lam = w[(size_t)t * m + j];
    const double2 *y = Y + ((size_t)t * m + j) * ne, *wv = W + ((size_t)t * m + j) * ne;
    double s = 0;
    for (int e = threadIdx.x; e < ne; e += kLB) {
        const double dr = wv[e].x - lam * y[e].x, di = wv[e].y - lam * y[e].y;
        s += dr * dr + di * di;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0;
        for (int q = 0; q < kLB / 64; ++q) tot += red[q];
        r2[(size_t)t * m + j] = tot;
    }
}

// ---- start block: a counter-based pseudo-random complex field per (t, j, e) -------------
__device__ __forceinline__ double hash_unit(unsigned long long k) {
    // splitmix64 finaliser, mapped to (-1, 1)
    k += 0x9E3779B97F4A7C15ull;
    k = (k ^ (k >> 30)) * 0xBF58476D1CE4E5B9ull;
    k = (k ^ (k >> 27)) * 0x94D049BB133111EBull;
    k ^= k >> 31;
    return (double)(k >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ __launch_bounds__(kLB) void start_kernel(double2 *X, int m, int ne, int lt) {
    const long idx = (long)blockIdx.x * kLB + threadIdx.x;
    const long total = (long)lt * m * ne;
    if (idx >= total) return;
    X[idx] = make_double2(hash_unit(2ull * (unsigned long long)idx), hash_unit(2ull * (unsigned long long)idx + 1));
}

// ---- phase convention and output -------------------------------------------------------
// The largest-modulus component real positive (the lowest canonical index 3 s + a
// among those within 1e-12 of the largest), then the vector is written to V[t][l]
// in the canonical order (element a vs + s of the block goes to 3 s + a).
__global__ __launch_bounds__(kLB) void phase_out_kernel(const double2 *Y, double2 *V, int m, int ne, int nev) {
    __shared__ double redd[kLB / 64];
    __shared__ int redi[kLB / 64];
    __shared__ double2 ph;
    const int l = blockIdx.x, t = blockIdx.y;
    const double2 *y = Y + ((size_t)t * m + l) * ne;
    double mx = 0;
    for (int e = threadIdx.x; e < ne; e += kLB) mx = fmax(mx, sqrt(y[e].x * y[e].x + y[e].y * y[e].y));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) redd[threadIdx.x >> 6] = mx;
    __syncthreads();
    mx = redd[0];
    for (int q = 1; q < kLB / 64; ++q) mx = fmax(mx, redd[q]);
    const int vs = ne / 3;
    int idx = ne;
    for (int e = threadIdx.x; e < ne; e += kLB) {
        const int ec = 3 * (e % vs) + e / vs;
        if (sqrt(y[e].x * y[e].x + y[e].y * y[e].y) >= mx - 1e-12 && ec < idx) idx = ec;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) idx = min(idx, __shfl_xor(idx, o, 64));
    if ((threadIdx.x & 63) == 0) redi[threadIdx.x >> 6] = idx;
    __syncthreads();
    if (threadIdx.x == 0) {
        int i = redi[0];
        for (int q = 1; q < kLB / 64; ++q) i = min(i, redi[q]);
        const double2 v = y[(i % 3) * vs + i / 3];
        const double a = sqrt(v.x * v.x + v.y * v.y);
        ph = a > 0 ? make_double2(v.x / a, -v.y / a) : make_double2(1, 0);   // conj(v) / |v|
    }
    __syncthreads();
    const double2 p = ph;
    double2 *out = V + ((size_t)t * nev + l) * ne;
    for (int e = threadIdx.x; e < ne; e += kLB) {
        const double2 v = y[(e % 3) * vs + e / 3];
        out[e] = make_double2(v.x * p.x - v.y * p.y, v.x * p.y + v.y * p.x);
    }
}

// ---- host side -----------------------------------------------------------------------------
struct EigWS {
    double2 *b[4];          // four blocks [lt][m][ne]
    double2 *C, *Q, *Z;     // [lt][m][m]
    double2 *gscratch;      // Gram partials
    double *w, *r2, *coef;  // [lt][m], [lt][m], [2][lt][3]
    int *flag;              // [lt] Cholesky breakdown flags
};

int eig_block(int nev) {
    int m = nev + (nev / 2 > 8 ? nev / 2 : 8);
    m += m & 1;
    return m > kEigMaxM ? kEigMaxM : m;
}

void gram_shape(int m, int ne, int lt, int &ntile, int &nsplit, int &nchunk) {
    (void)m;
    ntile = 1;   // one workgroup covers the whole block
    nchunk = (ne + kGKC - 1) / kGKC;
    const int base = lt;
    nsplit = (2048 + base - 1) / base;
    if (nsplit > nchunk) nsplit = nchunk;
    if (nsplit > 64) nsplit = 64;
    if (nsplit < 1) nsplit = 1;
}

size_t eig_layout(const Ctx &c, int nev, char *base, EigWS *ws) {
    const int m = eig_block(nev), lt = c.g.lt;
    const int ne = 3 * c.g.lx * c.g.ly * c.g.lz;
    int ntile, nsplit, nchunk;
    gram_shape(m, ne, lt, ntile, nsplit, nchunk);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += round256(bytes);
        return base ? base + o : nullptr;
    };
    EigWS w;
    for (int k = 0; k < 4; ++k) w.b[k] = reinterpret_cast<double2 *>(take((size_t)lt * m * ne * 16));
    w.C = reinterpret_cast<double2 *>(take((size_t)lt * m * m * 16));
    w.Q = reinterpret_cast<double2 *>(take((size_t)lt * m * m * 16));
    w.Z = reinterpret_cast<double2 *>(take((size_t)lt * m * m * 16));
    w.gscratch = reinterpret_cast<double2 *>(take((size_t)nsplit * lt * m * m * 16));
    w.w = reinterpret_cast<double *>(take((size_t)lt * m * 8));
    w.r2 = reinterpret_cast<double *>(take((size_t)lt * m * 8));
    w.coef = reinterpret_cast<double *>(take((size_t)lt * 6 * 8));
    w.flag = reinterpret_cast<int *>(take((size_t)lt * 4));
    if (ws) *ws = w;
    return off;
}

struct EigRun {
    const Ctx &c;
    EigWS ws;
    int m, ne, lt, vs;
    double chol_tiny;

    laph_status lap(const double2 *in, const double2 *z, double2 *out, const double *coef) const {
        LapArgs a;
        a.g = c.g;
        a.gp = c.gp;
        a.in = in;
        a.z = z;
        a.out = out;
        a.m = m;
        a.nvec = m;
        a.coef = coef;
        dim3 grid(((vs + kLapSites - 1) / kLapSites) * lt * ((m + LAPH_LAP_VG - 1) / LAPH_LAP_VG));
        if (a.z) hipLaunchKernelGGL((lap_kernel<true, true>), grid, dim3(kLB), 0, c.stream, a);
        else hipLaunchKernelGGL((lap_kernel<false, true>), grid, dim3(kLB), 0, c.stream, a);
        return check_launch("lap_kernel");
    }
    laph_status gram(const double2 *P, const double2 *R) const {
        GramArgs a;
        a.P = P;
        a.R = R;
        a.m = m;
        a.ne = ne;
        a.lt = lt;
        gram_shape(m, ne, lt, a.ntile, a.nsplit, a.nchunk);
        a.scratch = ws.gscratch;
        hipLaunchKernelGGL(gram_kernel, dim3(lt * a.nsplit), dim3(256), 0, c.stream, a);
        LAPH_TRY(check_launch("gram_kernel"));
        const long total = (long)lt * m * m;
        hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c.stream, a,
                           ws.C);
        return check_launch("gram_reduce_kernel");
    }
    laph_status jacobi(int mode, double shift_rel, int *only = nullptr) const {
        JacArgs a;
        a.C = ws.C;
        a.Q = ws.Q;
        a.Z = ws.Z;
        a.w = ws.w;
        a.m = m;
        a.mode = mode;
        a.shift_rel = shift_rel;
        a.max_sweeps = 40;
        a.flag = only;
        a.tiny = 0.0;
        hipLaunchKernelGGL(jacobi_kernel, dim3(lt), dim3(kJB), 0, c.stream, a);
        return check_launch("jacobi_kernel");
    }
    laph_status chol(double shift_rel) const {
        JacArgs a;
        a.C = ws.C;
        a.Q = ws.Q;
        a.Z = ws.Z;
        a.w = ws.w;
        a.m = m;
        a.mode = 1;
        a.shift_rel = shift_rel;
        a.max_sweeps = 0;
        a.flag = ws.flag;
        a.tiny = chol_tiny;
        hipLaunchKernelGGL(chol_kernel, dim3(lt), dim3(256), 0, c.stream, a);
        return check_launch("chol_kernel");
    }
    laph_status rotate(const double2 *in, double2 *out, bool tri = false) const {
        RotArgs a;
        a.in = in;
        a.out = out;
        a.Z = ws.Z;
        a.m = m;
        a.ne = ne;
        a.nout = m;
        a.mout = m;
        a.tri = tri ? ws.flag : nullptr;   // Cholesky's breakdown flags: 0 = triangular Z
        dim3 grid((ne + 4 * kRE - 1) / (4 * kRE), lt);
        hipLaunchKernelGGL(rotate_mfma_kernel, grid, dim3(256), 0, c.stream, a);
        return check_launch("rotate_mfma_kernel");
    }
};

}  // namespace

size_t laplacian_eig_workspace_bytes(const Ctx &c, int nev) { return eig_layout(c, nev, nullptr, nullptr); }

laph_status apply_neg_laplacian(const Ctx &c, double *out, const double *in, int nvec) {
    LapArgs a;
    a.g = c.g;
    a.gp = c.gp;
    a.in = reinterpret_cast<const double2 *>(in);
    a.z = nullptr;
    a.out = reinterpret_cast<double2 *>(out);
    a.m = nvec;
    a.nvec = nvec;
    a.coef = nullptr;
    const int vs = c.g.lx * c.g.ly * c.g.lz;
    dim3 grid(((vs + kLapSites - 1) / kLapSites) * c.g.lt * ((nvec + LAPH_LAP_VG - 1) / LAPH_LAP_VG));
    hipLaunchKernelGGL((lap_kernel<false, false>), grid, dim3(kLB), 0, c.stream, a);
    return check_launch("lap_kernel");
}

laph_status laplacian_eigvecs(Ctx &c, double *V, double *lam_host, int nev, double tol, int max_iter, int degree,
                              char *work, size_t bytes, int *iters_out, double *res_host) {
    const int m = eig_block(nev);
    if (nev < 1 || nev > 64 || m <= nev) return set_error(LAPH_ERR_INVALID, "nev must be in 1..64");
    if (!(tol > 0) || max_iter < 1) return set_error(LAPH_ERR_INVALID, "tol must be positive and max_iter >= 1");
    const size_t need = eig_layout(c, nev, nullptr, nullptr);
    if (!work || bytes < need) return set_error(LAPH_ERR_WORKSPACE, "workspace too small: %zu < %zu", bytes, need);
    // LAPH_EIG_CHOL_TINY overrides the Cholesky breakdown threshold (a value >= 1 sends
    // every timeslice through the eigendecomposition path)
    const char *tiny_env = std::getenv("LAPH_EIG_CHOL_TINY");
    const double tiny = tiny_env ? std::atof(tiny_env) : kCholTiny;
    EigRun R{c, {}, m, 3 * c.g.lx * c.g.ly * c.g.lz, c.g.lt, c.g.lx * c.g.ly * c.g.lz, tiny};
    eig_layout(c, nev, work, &R.ws);
    const int lt = R.lt, ne = R.ne;
    double2 *const *B = R.ws.b;
    // buffer roles by index into B: x = current block; the others are scratch
    int x = 0;
    auto other = [&](std::initializer_list<int> used) {
        for (int k = 0; k < 4; ++k) {
            bool u = false;
            for (int v : used) u |= v == k;
            if (!u) return k;
        }
        return -1;
    };
    // two orthonormalising passes Y <- Y R^{-1} (the first shifted; the second restores
    // orthonormality to rounding)
    auto loewdin = [&](int &cur) -> laph_status {
        for (int pass = 0; pass < 2; ++pass) {
            const int sp = other({cur});
            LAPH_TRY(R.gram(B[cur], B[cur]));
            const double shift = pass == 0 ? 1e-15 : 0.0;
            LAPH_TRY(R.chol(shift));
            LAPH_TRY(R.jacobi(1, shift, R.ws.flag));   // timeslices where Cholesky broke down
            LAPH_TRY(R.rotate(B[cur], B[sp], true));
            cur = sp;
        }
        return LAPH_OK;
    };
    {
        const long total = (long)lt * m * ne;
        hipLaunchKernelGGL(start_kernel, dim3((unsigned)((total + kLB - 1) / kLB)), dim3(kLB), 0, c.stream, B[x], m,
                           ne, lt);
        LAPH_TRY(check_launch("start_kernel"));
    }
    LAPH_TRY(loewdin(x));
    std::vector<double> cut(lt, 0.5 * kLmax), coef(6 * (size_t)lt), w((size_t)lt * m), r2((size_t)lt * m);
    const int deg_max = degree >= 2 ? degree : kDefaultDegree;
    std::vector<double> lo(lt, 0.0);   // lowest Ritz value per timeslice (-Delta >= 0 before the first)
    int it = 0;
    bool done = false;
    double worst = INFINITY;
    while (it < max_iter && !done) {
        ++it;
        // Chebyshev filter on [cut_t, 12]: Y1 = (A - c) X / e;  Y_{k+1} = 2 (A - c) Y_k / e - Y_{k-1}.
        // The degree is capped so that the filter grows the lowest Ritz direction by at
        // most ~1e6 over the cut (T_d(g) ~ e^{d acosh g} / 2): a larger ratio leaves the
        // block's other directions below rounding (the Gram matrix's condition is its square).
        int deg = deg_max;
        for (int t = 0; t < lt; ++t) {
            const double g = (0.5 * (cut[t] + kLmax) - lo[t]) / (0.5 * (kLmax - cut[t]));
            if (g > 1.0) deg = std::min(deg, std::max(2, (int)(std::log(2e6) / std::acosh(g))));
        }
        for (int t = 0; t < lt; ++t) {
            const double cc = 0.5 * (cut[t] + kLmax), ee = 0.5 * (kLmax - cut[t]);
            coef[3 * t] = 1.0 / ee;
            coef[3 * t + 1] = -cc / ee;
            coef[3 * t + 2] = 0.0;
            coef[3 * (lt + t)] = 2.0 / ee;
            coef[3 * (lt + t) + 1] = -2.0 * cc / ee;
            coef[3 * (lt + t) + 2] = -1.0;
        }
        LAPH_HIP(hipMemcpyAsync(R.ws.coef, coef.data(), coef.size() * 8, hipMemcpyHostToDevice, c.stream));
        // the copy reads the host vector asynchronously: wait before it can change
        LAPH_HIP(hipStreamSynchronize(c.stream));
        int prev = x, curr = other({x});
        LAPH_TRY(R.lap(B[prev], nullptr, B[curr], R.ws.coef));
        for (int k = 2; k <= deg; ++k) {
            const int next = other({prev, curr});
            LAPH_TRY(R.lap(B[curr], B[prev], B[next], R.ws.coef + 3 * lt));
            prev = curr;
            curr = next;
        }
        int blk = curr;
        LAPH_TRY(loewdin(blk));
        // Rayleigh-Ritz: H = Y^dagger (A Y); Ritz vectors Y Q and A Y Q; residual norms
        const int wb = other({blk});
        LAPH_TRY(R.lap(B[blk], nullptr, B[wb], nullptr));
        LAPH_TRY(R.gram(B[blk], B[wb]));
        LAPH_TRY(R.jacobi(0, 0.0));
        const int ry = other({blk, wb}), rw = other({blk, wb, ry});
        LAPH_TRY(R.rotate(B[blk], B[ry]));
        LAPH_TRY(R.rotate(B[wb], B[rw]));
        hipLaunchKernelGGL(residual_kernel, dim3(m, lt), dim3(kLB), 0, c.stream, B[ry], B[rw], R.ws.w, R.ws.r2, m, ne,
                           m);
        LAPH_TRY(check_launch("residual_kernel"));
        LAPH_HIP(hipMemcpyAsync(w.data(), R.ws.w, w.size() * 8, hipMemcpyDeviceToHost, c.stream));
        LAPH_HIP(hipMemcpyAsync(r2.data(), R.ws.r2, r2.size() * 8, hipMemcpyDeviceToHost, c.stream));
        LAPH_HIP(hipStreamSynchronize(c.stream));
        worst = 0;
        for (int t = 0; t < lt; ++t) {
            for (int j = 0; j < nev; ++j) worst = fmax(worst, sqrt(r2[(size_t)t * m + j]));
            cut[t] = w[(size_t)t * m + m - 1];
            lo[t] = w[(size_t)t * m];
        }
        if (!std::isfinite(worst)) return set_error(LAPH_ERR_NONFINITE, "non-finite residual in the eigensolver");
        done = worst <= tol;
        x = ry;   // the Ritz block starts the next iteration
    }
    if (iters_out) *iters_out = it;
    if (res_host) *res_host = worst;
    if (!done) return set_error(LAPH_ERR_NOCONV, "eigensolver did not reach tol in %d iterations", max_iter);
    hipLaunchKernelGGL(phase_out_kernel, dim3(nev, lt), dim3(kLB), 0, c.stream, B[x], reinterpret_cast<double2 *>(V),
                       m, ne, nev);
    LAPH_TRY(check_launch("phase_out_kernel"));
    for (int t = 0; t < lt; ++t)
        for (int j = 0; j < nev; ++j) lam_host[(size_t)t * nev + j] = w[(size_t)t * m + j];
    LAPH_HIP(hipStreamSynchronize(c.stream));
    return LAPH_OK;
}

}  // namespace laph
