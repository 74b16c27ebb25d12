// Meson doublets and baryon triplets of the LapH vectors (Sec. "QUDA": besides
// sourcing the solves and projecting the propagators, the LapH vectors form the
// quark-antiquark doublets and three-quark triplets that enter the Wick
// contractions of meson and baryon correlators).  Per timeslice t and momentum
// p = 2 pi (nx / Lx, ny / Ly, nz / Lz):
//
//   Phi_p[t][l][m]   = sum_x e^{-i p.x} sum_a conj(V_l(x, t)_a) V_m(x, t)_a
//   B_p[t][l][m][n]  = sum_x e^{-i p.x} eps_abc V_l(x, t)_a V_m(x, t)_b V_n(x, t)_c
//
// Both are complex FP64 GEMMs per (t, p) over K = (site, colour), 3 Lx Ly Lz long:
//   doublets  A[l][(x, a)] = e^{-i p.x} conj(V_l(x)_a),  B[(x, a)][m]      = V_m(x)_a
//   triplets  A[l][(x, a)] = e^{-i p.x} V_l(x)_a,        B[(x, a)][(m, n)] = (V_m(x) x V_n(x))_a
// where the triplet's B column is the colour cross product of a pair m < n.  A
// workgroup stages the V of a chunk of sites (all nev vectors) in LDS with the
// direct global-to-LDS loads, two chunks deep, so the next chunk arrives while the
// matrix cores work on the current one; each wave forms its A and B fragments from
// LDS (the cross products are never stored).  B_p is antisymmetric in every index pair, so
// only l < m < n is accumulated (a wave runs only the row blocks with some l below
// its pairs' largest m), and the reduction writes all six orderings with their signs and
// zeros where an index repeats.  K is split over workgroups for occupancy; the
// reduction sums the slices in a fixed order.
#include <algorithm>
#include <cmath>

#include "laph_solver.h"

namespace laph {

namespace {

constexpr int kCB = 256;          // threads per workgroup (4 waves)
constexpr int kCS = 8;            // sites per K chunk
constexpr int kCK = 3 * kCS;      // K (site, colour) per chunk
constexpr int kRS = kCK + 1;      // LDS row stride in complex (odd: conflict-free fragment reads)
constexpr int kSlots = 64 * kRS;  // complex slots of one staged chunk (64 rows)
constexpr int kCRows = 64;        // l rows: nev <= 64
constexpr int kCMaxMom = 16;      // momenta per launch
constexpr int kCTarget = 2048;    // workgroups aimed for by the K split

typedef double d4 __attribute__((ext_vector_type(4)));

struct ContractArgs {
    int lx, ly, lz, lt, vs;
    int nev;
    int ncol;             // doublets: nev; triplets: nev (nev - 1) / 2 pairs (m < n, m-major)
    int ntile;            // column tiles per (t, p)
    int nsplit;           // K slices
    int nchunk;           // K chunks of kCS sites
    int nmom;
    int mom[3 * kCMaxMom];
    const double2 *V;     // [lt][nev][vs][3]
    double2 *scratch;     // [nsplit][nmom][lt][nev][ncol]
};

// first column of pair row m in the m-major list of pairs m < n
__host__ __device__ __forceinline__ int pair_base(int m, int nev) { return m * nev - m * (m + 1) / 2; }

__device__ __forceinline__ void pair_of(int q, int nev, int &m, int &n) {
    m = 0;
    while (m + 1 < nev && pair_base(m + 1, nev) <= q) ++m;
    n = q - pair_base(m, nev) + m + 1;
}

// One staged chunk: the wave's A fragments (R row blocks) and B fragments (NCB column
// blocks) per group of 4 K, then the R x NCB x 4 real products as straight-line code,
// each product's accumulator written by the previous group's product of the same kind
// only (independent accumulators back to back).  A row of the chunk holds K colour-major
// (colour a of site s at a kCS + s), so with the 6 groups unrolled each group's colour
// and its cross-product partners are compile-time offsets from one per-lane address.
template <int MODE, int NCB, int R>
__device__ __forceinline__ void chunk_products(const double2 *buf, const double2 *ph, int lane, const int *cm,
                                               const int *cn, d4 (*cre)[NCB], d4 (*cim)[NCB]) {
    const int q = lane >> 4;   // K within a group of 4
    const double2 *arow = buf + (lane & 15) * kRS + q;
    const double2 *bm[NCB], *bn[NCB];
#pragma unroll
    for (int j = 0; j < NCB; ++j) {
        bm[j] = buf + cm[j] * kRS + q;
        bn[j] = buf + cn[j] * kRS + q;
    }
    // the phases of the two sites this lane meets (groups start at site 0 or 4)
    const double2 f0 = ph[q], f1 = ph[q + 4];
#pragma unroll
    for (int k4 = 0; k4 < kCK; k4 += 4) {
        const int a = k4 / kCS, so = k4 % kCS;   // colour and site offset of the group
        const double2 f = so ? f1 : f0;
        double ar[R], ai[R], nai[R], br[NCB], bi[NCB];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const double2 v = arow[16 * i * kRS + k4];
            const double vi = MODE == 0 ? -v.y : v.y;
            ar[i] = f.x * v.x - f.y * vi;
            ai[i] = f.x * vi + f.y * v.x;
            nai[i] = -ai[i];
        }
#pragma unroll
        for (int j = 0; j < NCB; ++j) {
            if (MODE == 0) {
                const double2 v = bm[j][k4];
                br[j] = v.x;
                bi[j] = v.y;
            } else {
                // (V_m x V_n)_a = V_m,b V_n,c - V_m,c V_n,b with (a, b, c) cyclic
                const int ob = (a == 2 ? 0 : a + 1) * kCS + so, oc = (a == 0 ? 2 : a - 1) * kCS + so;
                const double2 ub = bm[j][ob], uc = bm[j][oc];
                const double2 wb = bn[j][ob], wc = bn[j][oc];
                br[j] = (ub.x * wc.x - ub.y * wc.y) - (uc.x * wb.x - uc.y * wb.y);
                bi[j] = (ub.x * wc.y + ub.y * wc.x) - (uc.x * wb.y + uc.y * wb.x);
            }
        }
        // Re += Ar Br - Ai Bi;  Im += Ar Bi + Ai Br
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int j = 0; j < NCB; ++j) {
                cre[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], cre[i][j], 0, 0, 0);
                cim[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], cim[i][j], 0, 0, 0);
            }
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int j = 0; j < NCB; ++j) {
                cre[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai[i], bi[j], cre[i][j], 0, 0, 0);
                cim[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], cim[i][j], 0, 0, 0);
            }
        // keep each group's LDS reads with its products (hoisting them all costs occupancy)
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <int MODE, int NCB>
__device__ __forceinline__ void chunk_dispatch(int nact, const double2 *buf, const double2 *ph, int lane,
                                               const int *cm, const int *cn, d4 (*cre)[NCB], d4 (*cim)[NCB]) {
    switch (nact) {
        case 4: chunk_products<MODE, NCB, 4>(buf, ph, lane, cm, cn, cre, cim); break;
        case 3: chunk_products<MODE, NCB, 3>(buf, ph, lane, cm, cn, cre, cim); break;
        case 2: chunk_products<MODE, NCB, 2>(buf, ph, lane, cm, cn, cre, cim); break;
        case 1: chunk_products<MODE, NCB, 1>(buf, ph, lane, cm, cn, cre, cim); break;
        default: break;
    }
}

// Copy chunk s0 of every vector (64 rows, nev real) into LDS with the direct
// global-to-LDS loads: lane i of load q fills slot 64 q + i of the buffer, so each
// lane fetches the element that lands in its slot (which also reorders a row's K to
// colour-major).  Pad slots and rows or sites
// outside the data load the timeslice's first element (finite; the zero phase of a
// site outside the lattice cancels it, and pad slots and rows past nev are not read
// into any kept product).
__device__ __forceinline__ void stage_chunk(double2 *buf, const double2 *Vt, int nev, int n3, int s0, int wave,
                                            int lane) {
    for (int q = wave; q < kSlots / 64; q += 4) {
        const int e = 64 * q + lane;
        const int row = e / kRS, col = e - row * kRS;
        const int a = col / kCS, sl = col - a * kCS;   // colour-major within the row
        const double2 *src = Vt;
        if (col < kCK && row < nev && 3 * (s0 + sl) < n3) src = Vt + (size_t)row * n3 + 3 * (s0 + sl) + a;
        __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)(buf + 64 * q), 16, 0, 0);
    }
}

// NCB column blocks of 16 per wave: 4 NCB 16 columns per workgroup
template <int MODE, int NCB>
__global__ __launch_bounds__(kCB) void contract_kernel(ContractArgs A) {
    // two staged chunks: the next one is in flight while the products run on the other
    __shared__ double2 bufA[kSlots], bufB[kSlots];
    __shared__ double2 phA[kCS], phB[kCS];
    // workgroups that share a K slice of one timeslice run on one XCD (consecutive
    // workgroup ids go round-robin over the 8 XCDs)
    const int nb = gridDim.x;
    int bid = blockIdx.x;
    if (nb % 8 == 0) bid = (bid % 8) * (nb / 8) + bid / 8;
    const int inner = A.ntile * A.nmom;
    const int tile = bid % A.ntile;
    const int p = (bid / A.ntile) % A.nmom;
    const int outer = bid / inner;
    const int split = outer % A.nsplit;
    const int t = outer / A.nsplit;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int kCols = 4 * NCB * 16;
    const int nev = A.nev;

    // this lane's column per block, the pair behind it, and the number of 16-row
    // blocks the wave needs (wave-uniform: triplets need l < m, m at most the m of the
    // wave's last pair)
    int col[NCB], cm[NCB], cn[NCB];
    int rows_hi = 0;
#pragma unroll
    for (int j = 0; j < NCB; ++j) {
        const int c0 = tile * kCols + (wave * NCB + j) * 16;
        col[j] = c0 + (lane & 15);
        cm[j] = 0;
        cn[j] = 0;
        if (c0 >= A.ncol) continue;   // a block past the last column: zero B (V_0 x V_0, or column 0 unread)
        if (MODE == 1) {
            if (col[j] < A.ncol) pair_of(col[j], nev, cm[j], cn[j]);
            int mlast, nlast;
            pair_of(min(c0 + 15, A.ncol - 1), nev, mlast, nlast);
            rows_hi = max(rows_hi, mlast);
        } else {
            cm[j] = col[j] < A.ncol ? col[j] : 0;
            rows_hi = nev;
        }
    }
    const int nact = min(4, (rows_hi + 15) / 16);

    d4 cre[4][NCB], cim[4][NCB];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NCB; ++j) {
            cre[i][j] = d4{0, 0, 0, 0};
            cim[i][j] = d4{0, 0, 0, 0};
        }
    const int mx = A.mom[3 * p], my = A.mom[3 * p + 1], mz = A.mom[3 * p + 2];
    const int ch0 = (int)((long)A.nchunk * split / A.nsplit), ch1 = (int)((long)A.nchunk * (split + 1) / A.nsplit);
    const double2 *Vt = A.V + (size_t)t * nev * A.vs * 3;
    const int n3 = 3 * A.vs;
    // e^{-2 pi i (nx x / Lx + ny y / Ly + nz z / Lz)} of the chunk's sites, integer parts
    // reduced first; zero for sites past the timeslice
    auto phases = [&](double2 *ph, int s0) {
        if (tid < kCS) {
            const int s = s0 + tid;
            double2 v = make_double2(0.0, 0.0);
            if (s < A.vs) {
                const int x = s % A.lx, y = (s / A.lx) % A.ly, z = s / (A.lx * A.ly);
                const int qx = ((mx * x) % A.lx + A.lx) % A.lx;
                const int qy = ((my * y) % A.ly + A.ly) % A.ly;
                const int qz = ((mz * z) % A.lz + A.lz) % A.lz;
                const double f = (double)qx / A.lx + (double)qy / A.ly + (double)qz / A.lz;
                sincospi(-2.0 * f, &v.y, &v.x);
            }
            ph[tid] = v;
        }
    };
    if (ch0 < ch1) {
        stage_chunk(bufA, Vt, nev, n3, ch0 * kCS, wave, lane);
        phases(phA, ch0 * kCS);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int ch = ch0; ch < ch1; ch += 2) {
        if (ch + 1 < ch1) {
            stage_chunk(bufB, Vt, nev, n3, (ch + 1) * kCS, wave, lane);
            phases(phB, (ch + 1) * kCS);
        }
        chunk_dispatch<MODE, NCB>(nact, bufA, phA, lane, cm, cn, cre, cim);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (ch + 1 >= ch1) break;
        if (ch + 2 < ch1) {
            stage_chunk(bufA, Vt, nev, n3, (ch + 2) * kCS, wave, lane);
            phases(phA, (ch + 2) * kCS);
        }
        chunk_dispatch<MODE, NCB>(nact, bufB, phB, lane, cm, cn, cre, cim);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
    // v_mfma_f64_16x16x4f64 leaves C[row][col] of a 16 x 16 block in lane col + 16 (row % 4),
    // register row / 4 (a lane holds rows lane / 16 + 4 r of column lane % 16)
    double2 *out = A.scratch + (((size_t)split * A.nmom + p) * A.lt + t) * (size_t)nev * A.ncol;
#pragma unroll
    for (int j = 0; j < NCB; ++j) {
        if (col[j] >= A.ncol) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * i + (lane >> 4) + 4 * r;
                if (row < nev) out[(size_t)row * A.ncol + col[j]] = make_double2(cre[i][j][r], cim[i][j][r]);
            }
    }
}

// Phi[p][t][l][m] = sum over K slices
__global__ void doublet_reduce_kernel(ContractArgs A, double2 *phi, int p_begin, int nmom_total) {
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    const long per = (long)A.lt * A.nev * A.nev;
    if (idx >= per * A.nmom) return;
    const int p = (int)(idx / per);
    const long r = idx - p * per;
    double2 s = make_double2(0.0, 0.0);
    for (int sp = 0; sp < A.nsplit; ++sp) {
        const double2 v = A.scratch[((size_t)sp * A.nmom + p) * per + r];
        s.x += v.x;
        s.y += v.y;
    }
    (void)nmom_total;
    phi[(size_t)(p_begin + p) * per + r] = s;
}

// B[p][t][l][m][n]: the sum over K slices of the sorted triple's entry, with the
// sign of the permutation that sorts (l, m, n); zero when two indices coincide
__global__ void triplet_reduce_kernel(ContractArgs A, double2 *B, int p_begin) {
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    const int nev = A.nev;
    const long per = (long)A.lt * nev * nev * nev;
    if (idx >= per * A.nmom) return;
    const int p = (int)(idx / per);
    long r = idx - p * per;
    const int n = (int)(r % nev);
    const int m = (int)((r / nev) % nev);
    const int l = (int)((r / ((long)nev * nev)) % nev);
    const int t = (int)(r / ((long)nev * nev * nev));
    double2 s = make_double2(0.0, 0.0);
    if (l != m && m != n && l != n) {
        int a = l, b = m, c = n;
        double sg = 1.0;
        if (a > b) { int q = a; a = b; b = q; sg = -sg; }
        if (b > c) { int q = b; b = c; c = q; sg = -sg; }
        if (a > b) { int q = a; a = b; b = q; sg = -sg; }
        const int q = pair_base(b, nev) + (c - b - 1);
        for (int sp = 0; sp < A.nsplit; ++sp) {
            const double2 v = A.scratch[((((size_t)sp * A.nmom + p) * A.lt + t) * nev + a) * A.ncol + q];
            s.x += v.x;
            s.y += v.y;
        }
        s.x *= sg;
        s.y *= sg;
    }
    B[(size_t)(p_begin + p) * per + r] = s;
}

void contract_shape(const Ctx &c, int kind, int nev, int nmom, ContractArgs &a) {
    a.lx = c.g.lx;
    a.ly = c.g.ly;
    a.lz = c.g.lz;
    a.lt = c.g.lt;
    a.vs = c.g.lx * c.g.ly * c.g.lz;
    a.nev = nev;
    a.ncol = kind == 0 ? nev : nev * (nev - 1) / 2;
    const int cols = kind == 0 ? 64 : 128;
    a.ntile = std::max(1, (a.ncol + cols - 1) / cols);
    a.nmom = nmom;
    a.nchunk = (a.vs + kCS - 1) / kCS;
    const int base = a.lt * a.ntile * nmom;
    a.nsplit = std::max(1, std::min({(kCTarget + base - 1) / base, a.nchunk, 64}));
}

}  // namespace

// K-slice partials of one launch group of nmom momenta
static size_t group_bytes(const Ctx &c, int kind, int nev, int nmom) {
    ContractArgs a;
    contract_shape(c, kind, nev, nmom, a);
    return round256((size_t)a.nsplit * a.nmom * a.lt * nev * a.ncol * 16);
}

size_t contract_workspace_bytes(const Ctx &c, int kind, int nev, int n_mom) {
    if (nev < 1 || nev > kCRows || n_mom < 1 || (kind != 0 && kind != 1)) return 0;
    // the largest launch group: a full one, or the last (its K split may be finer)
    size_t b = group_bytes(c, kind, nev, std::min(n_mom, kCMaxMom));
    if (n_mom > kCMaxMom && n_mom % kCMaxMom) b = std::max(b, group_bytes(c, kind, nev, n_mom % kCMaxMom));
    return b;
}

laph_status contract(const Ctx &c, int kind, double *out, const double *V, int nev, int n_mom, const int *mom_host,
                     char *work, size_t bytes) {
    if (nev < 1 || nev > kCRows) return set_error(LAPH_ERR_INVALID, "nev must be in 1..%d", kCRows);
    if (kind == 1 && nev < 3) return set_error(LAPH_ERR_INVALID, "triplets need nev >= 3");
    if (n_mom < 1 || !mom_host) return set_error(LAPH_ERR_INVALID, "need at least one momentum");
    const size_t need = contract_workspace_bytes(c, kind, nev, n_mom);
    if (!work || bytes < need) return set_error(LAPH_ERR_WORKSPACE, "workspace too small: %zu < %zu", bytes, need);
    const size_t per = (size_t)c.g.lt * nev * nev * (kind == 0 ? 1 : nev);
    for (int p0 = 0; p0 < n_mom; p0 += kCMaxMom) {
        const int np = std::min(kCMaxMom, n_mom - p0);
        ContractArgs a;
        contract_shape(c, kind, nev, np, a);
        if (group_bytes(c, kind, nev, np) > bytes) return set_error(LAPH_ERR_WORKSPACE, "workspace too small");
        for (int q = 0; q < 3 * np; ++q) a.mom[q] = mom_host[3 * p0 + q];
        a.V = reinterpret_cast<const double2 *>(V);
        a.scratch = reinterpret_cast<double2 *>(work);
        const unsigned nblk = (unsigned)(a.lt * a.nsplit * a.ntile * a.nmom);
        if (kind == 0)
            hipLaunchKernelGGL((contract_kernel<0, 1>), dim3(nblk), dim3(kCB), 0, c.stream, a);
        else
            hipLaunchKernelGGL((contract_kernel<1, 2>), dim3(nblk), dim3(kCB), 0, c.stream, a);
        LAPH_TRY(check_launch("contract_kernel"));
        const long total = (long)per * np;
        const unsigned rb = (unsigned)((total + 255) / 256);
        if (kind == 0)
            hipLaunchKernelGGL(doublet_reduce_kernel, dim3(rb), dim3(256), 0, c.stream, a,
                               reinterpret_cast<double2 *>(out), p0, n_mom);
        else
            hipLaunchKernelGGL(triplet_reduce_kernel, dim3(rb), dim3(256), 0, c.stream, a,
                               reinterpret_cast<double2 *>(out), p0);
        LAPH_TRY(check_launch("contract_reduce_kernel"));
    }
    return LAPH_OK;
}

}  // namespace laph
