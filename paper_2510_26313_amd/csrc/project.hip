// LapH sources and the projection of solutions onto the LapH vectors.
//
// The projection is a complex FP64 GEMM per sink timeslice t,
//   C_t[l][(s, beta)] = sum_{(p, a, h)} conj(V_l(x, t)_a) X_s(x, t)_(beta, a),
// with M = nev, N = 4 * (RHS in the batch), K = 3 Lx Ly Lz.  The paper tiles
// this over (eigenvectors x solutions) so it fits memory (Sec. "Eigenvector
// Projection"); here a workgroup owns a 64 x 64 tile of C_t and a slice of K
// (split-K for occupancy), stages V and X through LDS and runs the FP64 matrix
// cores (v_mfma_f64_16x16x4f64); a second kernel sums the K slices in a fixed
// order and scatters into tau[t][l][k][beta][alpha].
#include "laph_solver.h"

namespace laph {

constexpr int kPB = 256;   // threads per projection workgroup (4 waves)
constexpr int kTM = 64;    // l per tile
constexpr int kTN = 64;    // (slot, beta) columns per tile
constexpr int kKC = 16;    // complex K per LDS stage
constexpr int kLd = kKC + 1;

typedef double d4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// sources
// ---------------------------------------------------------------------------
// Without noise (rho null) RHS r = 4k + alpha is V_k on spin alpha.  With noise, RHS
// r = 4j + alpha is the diluted noise source sum_{k = j mod n_dil} rho[alpha][k] V_k on
// spin alpha (interlaced LapH dilution, full spin and time dilution).
__device__ __forceinline__ cplx<double> source_colour(const double2 *V, const double2 *rho, int nev, int n_dil,
                                                      size_t v3, int t0, size_t site3, int r, int a) {
    const int kj = r >> 2, alpha = r & 3;
    if (!rho) {
        const double2 v = V[(((size_t)t0 * nev + kj) * v3 + site3) * 3 + a];
        return {v.x, v.y};
    }
    cplx<double> acc = {0.0, 0.0};
    for (int k = kj; k < nev; k += n_dil) {
        const double2 v = V[(((size_t)t0 * nev + k) * v3 + site3) * 3 + a];
        const double2 q = rho[(size_t)alpha * nev + k];
        acc.re += q.x * v.x - q.y * v.y;
        acc.im += q.x * v.y + q.y * v.x;
    }
    return acc;
}

__global__ void laph_sources_kernel(Geom g, Operand E, Operand O, const double2 *V, int nev, int t0, int r_begin,
                                    const double2 *rho, int n_dil, int p0, SiteWindow win) {
    const int h = blockIdx.x * 256 + threadIdx.x;
    const int s = blockIdx.y;
    const int p = p0 + blockIdx.z;
    if (h >= g.vh || !in_window(win, h, g.vh)) return;
    int x, y, z, t;
    site_coords(g, p, h, x, y, z, t);
    const int r = r_begin + s;
    const int alpha = r & 3;
    cplx<double> col[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    if (t == t0) {
        const size_t site3 = (size_t)x + (size_t)g.lx * (y + (size_t)g.ly * z);
        const size_t v3 = (size_t)g.lx * g.ly * g.lz;
#pragma unroll
        for (int a = 0; a < 3; ++a) col[a] = source_colour(V, rho, nev, n_dil, v3, t0, site3, r, a);
    }
    // spin alpha carries the colours (selected per component: a runtime index into the
    // spinor would put it in scratch memory)
    cplx<double> out[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) out[c] = (c / 3 == alpha) ? col[c % 3] : cplx<double>{0.0, 0.0};
    SpinorIO<F64>::store((p == 0 ? E : O).at(s), g.vh, h, out);
}

laph_status make_laph_sources(const Ctx &c, Operand E, Operand O, const double *V, int nev, int t0, int r_begin,
                              int n, const double *rho, int n_dil, int parity, SiteWindow win) {
    if (n <= 0) return LAPH_OK;
    dim3 grid((c.g.vh + 255) / 256, n, parity < 0 ? 2 : 1);
    hipLaunchKernelGGL(laph_sources_kernel, grid, dim3(256), 0, c.stream, c.g, E, O,
                       reinterpret_cast<const double2 *>(V), nev, t0, r_begin, reinterpret_cast<const double2 *>(rho),
                       n_dil, parity < 0 ? 0 : parity, win);
    return check_launch("laph_sources_kernel");
}

__global__ void sources_canonical_kernel(Geom g, double2 *B, const double2 *V, int nev, int t0, const double2 *rho,
                                         int n_dil) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    const long vol = 2L * g.vh;
    if (i >= vol) return;
    const long v3 = (long)g.lx * g.ly * g.lz;
    const int t = (int)(i / v3);
    const long site3 = i % v3;
    const int alpha = r & 3;
    double2 *dst = B + ((size_t)r * vol + i) * 12;
    for (int c = 0; c < 12; ++c) dst[c] = make_double2(0.0, 0.0);
    if (t == t0) {
        for (int a = 0; a < 3; ++a) {
            const cplx<double> v = source_colour(V, rho, nev, n_dil, (size_t)v3, t0, (size_t)site3, r, a);
            dst[3 * alpha + a] = make_double2(v.re, v.im);
        }
    }
}

laph_status make_sources_canonical(const Ctx &c, double *B, const double *V, int nev, int t0, const double *rho,
                                   int n_dil) {
    const long vol = 2L * c.g.vh;
    dim3 grid((unsigned)((vol + 255) / 256), 4 * (rho ? n_dil : nev));
    hipLaunchKernelGGL(sources_canonical_kernel, grid, dim3(256), 0, c.stream, c.g, reinterpret_cast<double2 *>(B),
                       reinterpret_cast<const double2 *>(V), nev, t0, reinterpret_cast<const double2 *>(rho), n_dil);
    return check_launch("sources_canonical_kernel");
}

// ---------------------------------------------------------------------------
// V in the internal site order: Vp[t][l][p][a][hh], hh = h - t * vs_h
// ---------------------------------------------------------------------------
size_t packed_v_bytes(const Ctx &c, int nev) { return round256((size_t)2 * c.g.vh * 3 * nev * 16); }

__global__ void pack_v_kernel(Geom g, double2 *Vp, const double2 *V, int nev) {
    const int h = blockIdx.x * 256 + threadIdx.x;
    const int l = blockIdx.y;
    const int p = blockIdx.z;
    if (h >= g.vh) return;
    int x, y, z, t;
    site_coords(g, p, h, x, y, z, t);
    const size_t v3 = (size_t)g.lx * g.ly * g.lz;
    const size_t site3 = (size_t)x + (size_t)g.lx * (y + (size_t)g.ly * z);
    const int hh = h - t * g.vs_h;
    const double2 *src = V + (((size_t)t * nev + l) * v3 + site3) * 3;
    double2 *dst = Vp + (((size_t)t * nev + l) * 2 + p) * 3 * (size_t)g.vs_h + hh;
    for (int a = 0; a < 3; ++a) dst[(size_t)a * g.vs_h] = src[a];
}

laph_status pack_laph_vectors(const Ctx &c, double *Vp, const double *V, int nev) {
    dim3 grid((c.g.vh + 255) / 256, nev, 2);
    hipLaunchKernelGGL(pack_v_kernel, grid, dim3(256), 0, c.stream, c.g, reinterpret_cast<double2 *>(Vp),
                       reinterpret_cast<const double2 *>(V), nev);
    return check_launch("pack_v_kernel");
}

// ---------------------------------------------------------------------------
// projection GEMM
// ---------------------------------------------------------------------------
struct ProjArgs {
    int vh, vs_h, lt;
    Operand xe, xo;
    int n;               // slots in the batch
    const double2 *Vp;
    int nev;
    int ntn;             // column tiles
    int nsplit;          // K slices
    int nchunk;          // K chunks of kKC per (p, a)
    double2 *scratch;    // [split][t][nev][N]
    int ncol;            // N = 4 n
};

__global__ __launch_bounds__(kPB) void project_kernel(ProjArgs A) {
    __shared__ double Vr[kTM][kLd], Vi[kTM][kLd], Xr[kTN][kLd], Xi[kTN][kLd];
    int bid = blockIdx.x;
    const int split = bid % A.nsplit;
    bid /= A.nsplit;
    const int tn = bid % A.ntn;
    const int t = bid / A.ntn;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    d4 cre[4], cim[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        cre[j] = d4{0, 0, 0, 0};
        cim[j] = d4{0, 0, 0, 0};
    }
    // K = 6 * nchunk chunks in (p, a, hh-chunk) order; this slice takes a contiguous range
    const int total = 6 * A.nchunk;
    const int c0 = (int)((long)total * split / A.nsplit), c1 = (int)((long)total * (split + 1) / A.nsplit);
    const int krow = tid & 15;   // k within the chunk for the loaders
    const int rsub = tid >> 4;   // 0..15
    for (int ch = c0; ch < c1; ++ch) {
        const int pa = ch / A.nchunk;          // p * 3 + a
        const int hh0 = (ch - pa * A.nchunk) * kKC;
        const int p = pa / 3, a = pa - 3 * (pa / 3);
        const int hh = hh0 + krow;
        const bool kin = hh < A.vs_h;
        // V tile: rows l, this chunk's K
#pragma unroll
        for (int j = 0; j < kTM / 16; ++j) {
            const int l = rsub + 16 * j;
            double2 v = make_double2(0, 0);
            if (kin && l < A.nev) v = A.Vp[(((size_t)t * A.nev + l) * 6 + pa) * A.vs_h + hh];
            Vr[l][krow] = v.x;
            Vi[l][krow] = v.y;
        }
        // X tile: columns (slot, beta) of this column tile
#pragma unroll
        for (int j = 0; j < kTN / 16; ++j) {
            const int col = rsub + 16 * j;
            const int gcol = tn * kTN + col;
            const int s = gcol >> 2, beta = gcol & 3;
            double2 x = make_double2(0, 0);
            if (kin && s < A.n) {
                const char *hv = (p == 0 ? A.xe : A.xo).at(s);
                x = reinterpret_cast<const double2 *>(hv)[(size_t)(3 * beta + a) * A.vh + (size_t)t * A.vs_h + hh];
            }
            Xr[col][krow] = x.x;
            Xi[col][krow] = x.y;
        }
        __syncthreads();
#pragma unroll
        for (int k4 = 0; k4 < kKC; k4 += 4) {
            const int arow = wave * 16 + (lane & 15);
            const int kk = k4 + (lane >> 4);
            const double ar = Vr[arow][kk], ai = Vi[arow][kk];
            const double nai = -ai;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int bcol = j * 16 + (lane & 15);
                const double br = Xr[bcol][kk], bi = Xi[bcol][kk];
                // conj(V) X = (Vr Xr + Vi Xi) + i (Vr Xi - Vi Xr)
                cre[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, cre[j], 0, 0, 0);
                cre[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, cre[j], 0, 0, 0);
                cim[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, cim[j], 0, 0, 0);
                cim[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai, br, cim[j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // write this slice's partial C tile: v_mfma_f64_16x16x4f64 leaves C[row][col] in lane
    // col + 16 * (row % 4), register row / 4 (lane holds rows lane/16 + 4 i, column lane%16)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int gcol = tn * kTN + j * 16 + (lane & 15);
        if (gcol >= A.ncol) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int l = wave * 16 + (lane >> 4) + 4 * i;
            if (l >= A.nev) continue;
            A.scratch[(((size_t)split * A.lt + t) * A.nev + l) * A.ncol + gcol] = make_double2(cre[j][i], cim[j][i]);
        }
    }
}

// tau[t][l][k][beta][alpha] = sum over slices, RHS r = r_begin + s = 4k + alpha
__global__ void project_reduce_kernel(ProjArgs A, double2 *tau, int nev_src, int r_begin) {
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    const long total = (long)A.lt * A.nev * A.ncol;
    if (idx >= total) return;
    const int gcol = (int)(idx % A.ncol);
    const int l = (int)((idx / A.ncol) % A.nev);
    const int t = (int)(idx / ((long)A.ncol * A.nev));
    double2 s = make_double2(0, 0);
    for (int sp = 0; sp < A.nsplit; ++sp) {
        double2 v = A.scratch[(((size_t)sp * A.lt + t) * A.nev + l) * A.ncol + gcol];
        s.x += v.x;
        s.y += v.y;
    }
    const int slot = gcol >> 2, beta = gcol & 3;
    const int r = r_begin + slot;
    const int k = r >> 2, alpha = r & 3;
    tau[((((size_t)t * A.nev + l) * nev_src + k) * 4 + beta) * 4 + alpha] = s;
}

static void proj_shape(const Ctx &c, int nev, int n, int &ntn, int &nsplit, int &nchunk) {
    ntn = (4 * n + kTN - 1) / kTN;
    nchunk = (c.g.vs_h + kKC - 1) / kKC;
    const int base = c.g.lt * ntn * ((nev + kTM - 1) / kTM);
    nsplit = (2048 + base - 1) / base;
    if (nsplit > 6 * nchunk) nsplit = 6 * nchunk;
    if (nsplit > 64) nsplit = 64;
    if (nsplit < 1) nsplit = 1;
}

size_t project_scratch_bytes(const Ctx &c, int nev, int n) {
    int ntn, nsplit, nchunk;
    proj_shape(c, nev, n, ntn, nsplit, nchunk);
    return round256((size_t)nsplit * c.g.lt * nev * 4 * n * 16);
}

laph_status project(const Ctx &c, const ProjectSpec &s) {
    if (s.n <= 0) return LAPH_OK;
    if (s.nev > kTM) return set_error(LAPH_ERR_INVALID, "projection supports nev <= %d", kTM);
    ProjArgs a;
    a.vh = c.g.vh;
    a.vs_h = c.g.vs_h;
    a.lt = c.g.lt;
    a.xe = s.xe;
    a.xo = s.xo;
    a.n = s.n;
    a.Vp = reinterpret_cast<const double2 *>(s.Vp);
    a.nev = s.nev;
    proj_shape(c, s.nev, s.n, a.ntn, a.nsplit, a.nchunk);
    a.scratch = reinterpret_cast<double2 *>(s.scratch);
    a.ncol = 4 * s.n;
    const int nblk = c.g.lt * a.ntn * a.nsplit;
    hipLaunchKernelGGL(project_kernel, dim3(nblk), dim3(kPB), 0, c.stream, a);
    LAPH_TRY(check_launch("project_kernel"));
    const long total = (long)c.g.lt * s.nev * a.ncol;
    hipLaunchKernelGGL(project_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c.stream, a,
                       reinterpret_cast<double2 *>(s.tau), s.nev_src, s.r_begin);
    return check_launch("project_reduce_kernel");
}

// ---------------------------------------------------------------------------
// spin basis: tau' = S tau S^dagger on every 4 x 4 (sink spin, source spin) block
// (a change of Dirac basis psi' = S psi; the paper's driver adds such a basis)
// ---------------------------------------------------------------------------
struct SpinMat {
    double2 s[16];   // S[row][col], row-major
};

__global__ void spin_rotate_kernel(double2 *out, const double2 *tau, long nblk, SpinMat S) {
    const long b = (long)blockIdx.x * 256 + threadIdx.x;
    if (b >= nblk) return;
    cplx<double> m[16], sm[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) m[i] = {tau[b * 16 + i].x, tau[b * 16 + i].y};
    // sm = S m
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            cplx<double> acc = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 4; ++k) cmac(acc, cplx<double>{S.s[4 * r + k].x, S.s[4 * r + k].y}, m[4 * k + c]);
            sm[4 * r + c] = acc;
        }
    // out = sm S^dagger: out[r][c] = sum_k sm[r][k] conj(S[c][k])
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            cplx<double> acc = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 4; ++k) cmac_conj(acc, cplx<double>{S.s[4 * c + k].x, S.s[4 * c + k].y}, sm[4 * r + k]);
            out[b * 16 + 4 * r + c] = make_double2(acc.re, acc.im);
        }
}

laph_status spin_rotate(const Ctx &c, double *out, const double *tau, long nblk, const double *S_host) {
    if (nblk <= 0) return LAPH_OK;
    SpinMat S;
    for (int i = 0; i < 16; ++i) S.s[i] = make_double2(S_host[2 * i], S_host[2 * i + 1]);
    hipLaunchKernelGGL(spin_rotate_kernel, dim3((unsigned)((nblk + 255) / 256)), dim3(256), 0, c.stream,
                       reinterpret_cast<double2 *>(out), reinterpret_cast<const double2 *>(tau), nblk, S);
    return check_launch("spin_rotate_kernel");
}

// ---------------------------------------------------------------------------
// adjoint of the projection: GX^(4k+alpha)(x, t)_(beta, a) = sum_l V_l(x, t)_a Gtau[t][l][k][beta][alpha]
// ---------------------------------------------------------------------------
__global__ void project_adjoint_kernel(Geom g, double2 *GX, const double2 *Gtau, const double2 *V, int nev,
                                       int nev_src) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    const long vol = 2L * g.vh;
    if (i >= vol) return;
    const long v3 = (long)g.lx * g.ly * g.lz;
    const int t = (int)(i / v3);
    const long site3 = i % v3;
    const int k = r >> 2, alpha = r & 3;
    double2 *dst = GX + ((size_t)r * vol + i) * 12;
    for (int beta = 0; beta < 4; ++beta)
        for (int a = 0; a < 3; ++a) {
            double re = 0, im = 0;
            for (int l = 0; l < nev; ++l) {
                const double2 v = V[(((size_t)t * nev + l) * v3 + site3) * 3 + a];
                const double2 gt = Gtau[((((size_t)t * nev + l) * nev_src + k) * 4 + beta) * 4 + alpha];
                re += v.x * gt.x - v.y * gt.y;
                im += v.x * gt.y + v.y * gt.x;
            }
            dst[3 * beta + a] = make_double2(re, im);
        }
}

laph_status project_adjoint(const Ctx &c, double *GX, const double *Gtau, const double *V, int nev, int nev_src) {
    const long vol = 2L * c.g.vh;
    dim3 grid((unsigned)((vol + 255) / 256), 4 * nev_src);
    hipLaunchKernelGGL(project_adjoint_kernel, grid, dim3(256), 0, c.stream, c.g, reinterpret_cast<double2 *>(GX),
                       reinterpret_cast<const double2 *>(Gtau), reinterpret_cast<const double2 *>(V), nev, nev_src);
    return check_launch("project_adjoint_kernel");
}

}  // namespace laph
