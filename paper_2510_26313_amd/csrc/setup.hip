// Setup kernels: gauge ingest (canonical -> even-odd SoA in FP64 / FP32 / FP16,
// SU(3) check), clover term and the Cholesky-based inverses of its chiral blocks
// (FP64), and spinor pack / unpack between the canonical and internal layouts.
#include <cstring>

#include "laph_host.h"

namespace laph {

constexpr int kSetupBlock = 256;

// 3x3 complex matrices in FP64 for the clover construction
struct M3 {
    cplx<double> m[9];
};
__device__ __forceinline__ M3 mmul(const M3 &a, const M3 &b) {
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cplx<double> s = {0, 0};
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac(s, a.m[i * 3 + k], b.m[k * 3 + j]);
            c.m[i * 3 + j] = s;
        }
    return c;
}
__device__ __forceinline__ M3 adj(const M3 &a) {
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) c.m[i * 3 + j] = conj(a.m[j * 3 + i]);
    return c;
}
__device__ __forceinline__ M3 madd(const M3 &a, const M3 &b) {
    M3 c;
#pragma unroll
    for (int k = 0; k < 9; ++k) c.m[k] = a.m[k] + b.m[k];
    return c;
}

// ---------------------------------------------------------------------------
// gauge ingest
// ---------------------------------------------------------------------------
__global__ void gauge_pack_kernel(Geom g, const double2 *U, GaugePtrs gp, unsigned long long *maxdev) {
    const long i = (long)blockIdx.x * kSetupBlock + threadIdx.x;
    const long vol = 2L * g.vh;
    if (i >= vol) return;
    const int x = (int)(i % g.lx);
    const int y = (int)((i / g.lx) % g.ly);
    const int z = (int)((i / ((long)g.lx * g.ly)) % g.lz);
    const int t = (int)(i / ((long)g.lx * g.ly * g.lz));
    const int p = (x + y + z + t) & 1;
    const int h = (int)(i >> 1);
    double dev = 0;
    for (int mu = 0; mu < 4; ++mu) {
        cplx<double> u[9];
        for (int k = 0; k < 9; ++k) {
            double2 v = U[(i * 4 + mu) * 9 + k];
            u[k] = {v.x, v.y};
        }
        // distance from SU(3): |U U^+ - 1| and |det U - 1|
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                cplx<double> s = {a == b ? -1.0 : 0.0, 0.0};
                for (int k = 0; k < 3; ++k) cmac_conj(s, u[b * 3 + k], u[a * 3 + k]);
                dev = fmax(dev, fmax(fabs(s.re), fabs(s.im)));
            }
        cplx<double> det = u[0] * (u[4] * u[8] - u[5] * u[7]) - u[1] * (u[3] * u[8] - u[5] * u[6]) +
                           u[2] * (u[3] * u[7] - u[4] * u[6]);
        dev = fmax(dev, fmax(fabs(det.re - 1.0), fabs(det.im)));
        double2 *d64 = reinterpret_cast<double2 *>(const_cast<char *>(gp.f64[p][mu]));
        for (int k = 0; k < 9; ++k) d64[(size_t)k * g.vh + h] = make_double2(u[k].re, u[k].im);
        float4 *d32 = reinterpret_cast<float4 *>(const_cast<char *>(gp.f32[p][mu]));
        for (int j = 0; j < 3; ++j)
            d32[(size_t)j * g.vh + h] = make_float4((float)u[2 * j].re, (float)u[2 * j].im,
                                                    (float)u[2 * j + 1].re, (float)u[2 * j + 1].im);
        half8 a8;
        for (int k = 0; k < 4; ++k) {
            a8[2 * k] = (_Float16)u[k].re;
            a8[2 * k + 1] = (_Float16)u[k].im;
        }
        half4 b4;
        b4[0] = (_Float16)u[4].re;
        b4[1] = (_Float16)u[4].im;
        b4[2] = (_Float16)u[5].re;
        b4[3] = (_Float16)u[5].im;
        reinterpret_cast<half8 *>(const_cast<char *>(gp.f16a[p][mu]))[h] = a8;
        reinterpret_cast<half4 *>(const_cast<char *>(gp.f16b[p][mu]))[h] = b4;
    }
    if (!(dev <= 1e300)) dev = 1e300;  // NaN -> huge
    atomicMax(maxdev, (unsigned long long)__double_as_longlong(dev));
}

laph_status load_gauge(Ctx &c, const double *U) {
    unsigned long long *d_max = c.gauge_dev();
    LAPH_HIP(hipMemsetAsync(d_max, 0, sizeof(unsigned long long), c.stream));
    const long vol = 2L * c.g.vh;
    hipLaunchKernelGGL(gauge_pack_kernel, dim3((unsigned)((vol + kSetupBlock - 1) / kSetupBlock)), dim3(kSetupBlock),
                       0, c.stream, c.g, reinterpret_cast<const double2 *>(U), c.gp, d_max);
    LAPH_TRY(check_launch("gauge_pack_kernel"));
    unsigned long long hmax = 0;
    LAPH_HIP(hipMemcpyAsync(&hmax, d_max, sizeof(hmax), hipMemcpyDeviceToHost, c.stream));
    LAPH_HIP(hipStreamSynchronize(c.stream));
    double dev;
    memcpy(&dev, &hmax, sizeof(dev));
    if (!(dev <= 1e-10)) {
        c.gauge_loaded = false;
        return set_error(LAPH_ERR_INVALID, "gauge field is not SU(3): max deviation %.3e > 1e-10", dev);
    }
    c.gauge_loaded = true;
    c.n_mass = 0;
    return LAPH_OK;
}

// ---------------------------------------------------------------------------
// clover term
// ---------------------------------------------------------------------------
__device__ __forceinline__ M3 link64(const Geom &g, const GaugePtrs &gp, int x, int y, int z, int t, int mu) {
    x = (x + g.lx) % g.lx;
    y = (y + g.ly) % g.ly;
    z = (z + g.lz) % g.lz;
    t = (t + g.lt) % g.lt;
    const int p = (x + y + z + t) & 1;
    const int h = cb_index(g, x, y, z, t);
    M3 u;
    GaugeIO<F64>::load(gp, p, mu, g.vh, h, u.m);
    return u;
}

// F_munu(x) = (Q - Q^+)/8 minus its trace part, Q = sum of the four plaquettes at x
__device__ M3 field_strength(const Geom &g, const GaugePtrs &gp, const int (&x)[4], int mu, int nu) {
    auto at = [&](int dm, int dn, int dir) {
        int c[4] = {x[0], x[1], x[2], x[3]};
        c[mu] += dm;
        c[nu] += dn;
        return link64(g, gp, c[0], c[1], c[2], c[3], dir);
    };
    M3 q;
    // x -> x+mu -> x+mu+nu -> x+nu -> x
    q = mmul(mmul(at(0, 0, mu), at(1, 0, nu)), mmul(adj(at(0, 1, mu)), adj(at(0, 0, nu))));
    // x -> x+nu -> x+nu-mu -> x-mu -> x
    q = madd(q, mmul(mmul(at(0, 0, nu), adj(at(-1, 1, mu))), mmul(adj(at(-1, 0, nu)), at(-1, 0, mu))));
    // x -> x-mu -> x-mu-nu -> x-nu -> x
    q = madd(q, mmul(mmul(adj(at(-1, 0, mu)), adj(at(-1, -1, nu))), mmul(at(-1, -1, mu), at(0, -1, nu))));
    // x -> x-nu -> x-nu+mu -> x+mu -> x
    q = madd(q, mmul(mmul(adj(at(0, -1, nu)), at(0, -1, mu)), mmul(at(1, -1, nu), adj(at(0, 0, mu)))));
    M3 f;
    cplx<double> tr = {0, 0};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            f.m[i * 3 + j] = 0.125 * (q.m[i * 3 + j] - conj(q.m[j * 3 + i]));
            if (i == j) tr = tr + f.m[i * 3 + j];
        }
#pragma unroll
    for (int i = 0; i < 3; ++i) f.m[i * 4] = f.m[i * 4] - (1.0 / 3.0) * tr;
    return f;
}

// Packed Hermitian clover term per site and chiral block (without 4 + m0):
// in this gamma basis sigma_munu is block diagonal; on spins {0,1} (block 0)
//   sum sigma (x) F = sx (x) (Fyz - Fxt) + sy (x) (Fxz + Fyt) + sz (x) (Fxy - Fzt)
// and on spins {2,3} (block 1) the signs of the time planes flip, with
// sx, sy, sz the Pauli matrices.  The block is (i/2) c_sw times that sum.
__global__ void clover_build_kernel(Geom g, GaugePtrs gp, double csw, char *term0, char *term1) {
    const int h = blockIdx.x * kSetupBlock + threadIdx.x;
    const int p = blockIdx.y;
    if (h >= g.vh) return;
    int x[4];
    site_coords(g, p, h, x[0], x[1], x[2], x[3]);
    M3 Fxy = field_strength(g, gp, x, 0, 1), Fxz = field_strength(g, gp, x, 0, 2);
    M3 Fyz = field_strength(g, gp, x, 1, 2), Fxt = field_strength(g, gp, x, 0, 3);
    M3 Fyt = field_strength(g, gp, x, 1, 3), Fzt = field_strength(g, gp, x, 2, 3);
    double2 *dst = reinterpret_cast<double2 *>(p == 0 ? term0 : term1);
    for (int blk = 0; blk < 2; ++blk) {
        const double sgn = blk == 0 ? -1.0 : 1.0;
        cplx<double> Gx[9], Gy[9], Gz[9];
        const cplx<double> ihalf = {0.0, 0.5 * csw};
        for (int k = 0; k < 9; ++k) {
            Gx[k] = ihalf * (Fyz.m[k] + sgn * Fxt.m[k]);
            Gy[k] = ihalf * (Fxz.m[k] - sgn * Fyt.m[k]);
            Gz[k] = ihalf * (Fxy.m[k] + sgn * Fzt.m[k]);
        }
        // 6x6 = [[Gz, Gx - i Gy], [Gx + i Gy, -Gz]], index 3 s' + a
        double pk[36];
        auto entry = [&](int i, int j) -> cplx<double> {
            const int si = i / 3, a = i % 3, sj = j / 3, b = j % 3;
            const int k = a * 3 + b;
            if (si == 0 && sj == 0) return Gz[k];
            if (si == 1 && sj == 1) return cplx<double>{-Gz[k].re, -Gz[k].im};
            if (si == 1 && sj == 0) return Gx[k] + mul_i(Gy[k]);
            return Gx[k] - mul_i(Gy[k]);
        };
        for (int i = 0; i < 6; ++i) pk[i] = entry(i, i).re;
        int k = 0;
        for (int i = 1; i < 6; ++i)
            for (int j = 0; j < i; ++j) {
                cplx<double> e = entry(i, j);
                pk[6 + 2 * k] = e.re;
                pk[7 + 2 * k] = e.im;
                ++k;
            }
        double2 *d = dst + (size_t)blk * 18 * g.vh;
        for (int q = 0; q < 18; ++q) d[(size_t)q * g.vh + h] = make_double2(pk[2 * q], pk[2 * q + 1]);
    }
}

// Inverse of (term + shift) per site and block by Cholesky: A = L L^+, A^-1 = W^+ W, W = L^-1.
__global__ void clover_invert_kernel(int vh, const char *term, double shift, char *inv64, char *inv32, int *bad) {
    const int h = blockIdx.x * kSetupBlock + threadIdx.x;
    const int blk = blockIdx.y;
    if (h >= vh) return;
    double m[36];
    CloverIO<F64>::load(term, blk, vh, h, m);
    cplx<double> A[6][6];
    int k = 0;
    for (int i = 0; i < 6; ++i) A[i][i] = {m[i] + shift, 0.0};
    for (int i = 1; i < 6; ++i)
        for (int j = 0; j < i; ++j) {
            A[i][j] = {m[6 + 2 * k], m[7 + 2 * k]};
            A[j][i] = conj(A[i][j]);
            ++k;
        }
    cplx<double> Lm[6][6];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) Lm[i][j] = {0, 0};
    bool ok = true;
    for (int j = 0; j < 6; ++j) {
        double d = A[j][j].re;
        for (int q = 0; q < j; ++q) d -= Lm[j][q].re * Lm[j][q].re + Lm[j][q].im * Lm[j][q].im;
        if (!(d > 0)) {
            ok = false;
            d = 1.0;
        }
        const double ljj = sqrt(d);
        Lm[j][j] = {ljj, 0};
        for (int i = j + 1; i < 6; ++i) {
            cplx<double> s = A[i][j];
            for (int q = 0; q < j; ++q) {
                // s -= L[i][q] conj(L[j][q])
                cplx<double> t = Lm[i][q] * conj(Lm[j][q]);
                s = s - t;
            }
            Lm[i][j] = (1.0 / ljj) * s;
        }
    }
    if (!ok) atomicOr(bad, 1);
    // W = L^-1 (lower triangular)
    cplx<double> W[6][6];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) W[i][j] = {0, 0};
    for (int j = 0; j < 6; ++j) {
        W[j][j] = {1.0 / Lm[j][j].re, 0};
        for (int i = j + 1; i < 6; ++i) {
            cplx<double> s = {0, 0};
            for (int q = j; q < i; ++q) cmac(s, Lm[i][q], W[q][j]);
            W[i][j] = (-1.0 / Lm[i][i].re) * s;
        }
    }
    // A^-1 = W^+ W: (i, j) = sum_{q >= max(i,j)} conj(W[q][i]) W[q][j]
    double out[36];
    for (int i = 0; i < 6; ++i) {
        double s = 0;
        for (int q = i; q < 6; ++q) s += W[q][i].re * W[q][i].re + W[q][i].im * W[q][i].im;
        out[i] = s;
    }
    k = 0;
    for (int i = 1; i < 6; ++i)
        for (int j = 0; j < i; ++j) {
            cplx<double> s = {0, 0};
            for (int q = i; q < 6; ++q) cmac_conj(s, W[q][i], W[q][j]);
            out[6 + 2 * k] = s.re;
            out[7 + 2 * k] = s.im;
            ++k;
        }
    double2 *d64 = reinterpret_cast<double2 *>(inv64) + (size_t)blk * 18 * vh;
    for (int q = 0; q < 18; ++q) d64[(size_t)q * vh + h] = make_double2(out[2 * q], out[2 * q + 1]);
    float4 *d32 = reinterpret_cast<float4 *>(inv32) + (size_t)blk * 9 * vh;
    for (int q = 0; q < 9; ++q)
        d32[(size_t)q * vh + h] = make_float4((float)out[4 * q], (float)out[4 * q + 1], (float)out[4 * q + 2],
                                              (float)out[4 * q + 3]);
}

laph_status build_clover(Ctx &c, double csw, int n_mass, const double *m0) {
    char *t0 = c.state + c.off_clov;
    char *t1 = t0 + c.sz_cl64_par;
    dim3 grid((c.g.vh + kSetupBlock - 1) / kSetupBlock, 2);
    hipLaunchKernelGGL(clover_build_kernel, grid, dim3(kSetupBlock), 0, c.stream, c.g, c.gp, csw, t0, t1);
    LAPH_TRY(check_launch("clover_build_kernel"));
    double *diag = c.mass_diag();
    int *d_bad = c.bad_flag();
    LAPH_HIP(hipMemsetAsync(d_bad, 0, sizeof(int), c.stream));
    std::vector<double> hdiag(n_mass);
    for (int m = 0; m < n_mass; ++m) {
        hdiag[m] = 4.0 + m0[m];
        for (int p = 0; p < 2; ++p) {
            dim3 gi((c.g.vh + kSetupBlock - 1) / kSetupBlock, 2);
            hipLaunchKernelGGL(clover_invert_kernel, gi, dim3(kSetupBlock), 0, c.stream, c.g.vh,
                               (const char *)c.clover_term(p), 4.0 + m0[m], const_cast<char *>(c.clover_inv64(m, p)),
                               const_cast<char *>(c.clover_inv32(m, p)), d_bad);
            LAPH_TRY(check_launch("clover_invert_kernel"));
        }
    }
    LAPH_HIP(hipMemcpyAsync(diag, hdiag.data(), n_mass * sizeof(double), hipMemcpyHostToDevice, c.stream));
    int hbad = 0;
    LAPH_HIP(hipMemcpyAsync(&hbad, d_bad, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    LAPH_HIP(hipStreamSynchronize(c.stream));
    if (hbad) {
        c.n_mass = 0;
        return set_error(LAPH_ERR_INVALID, "clover block not positive definite (4 + m0 too small?)");
    }
    c.n_mass = n_mass;
    c.csw = csw;
    c.m0.assign(m0, m0 + n_mass);
    return LAPH_OK;
}

// ---------------------------------------------------------------------------
// spinor pack / unpack
// ---------------------------------------------------------------------------
template <class P>
__global__ void pack_kernel(Geom g, Operand out, const double2 *in, size_t in_rhs_stride, int parity, int nparity) {
    using R = typename P::real;
    const int h = blockIdx.x * kSetupBlock + threadIdx.x;
    const int r = blockIdx.y;
    const int pi = blockIdx.z;
    if (h >= g.vh) return;
    const int p = nparity == 2 ? pi : parity;
    int x, y, z, t;
    site_coords(g, p, h, x, y, z, t);
    const size_t i = (size_t)x + (size_t)g.lx * (y + (size_t)g.ly * (z + (size_t)g.lz * t));
    const double2 *src = in + r * in_rhs_stride + i * 12;
    cplx<R> s[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        double2 v = src[c];
        s[c] = {R(v.x), R(v.y)};
    }
    char *hv = out.at(r) + (nparity == 2 ? pi * (out.stride / 2) : 0);
    SpinorIO<P>::store(hv, g.vh, h, s);
}

template <class P>
__global__ void unpack_kernel(Geom g, double2 *out, size_t out_rhs_stride, Operand in, int parity, int nparity) {
    using R = typename P::real;
    const int h = blockIdx.x * kSetupBlock + threadIdx.x;
    const int r = blockIdx.y;
    const int pi = blockIdx.z;
    if (h >= g.vh) return;
    const int p = nparity == 2 ? pi : parity;
    int x, y, z, t;
    site_coords(g, p, h, x, y, z, t);
    const size_t i = (size_t)x + (size_t)g.lx * (y + (size_t)g.ly * (z + (size_t)g.lz * t));
    const char *hv = in.at(r) + (nparity == 2 ? pi * (in.stride / 2) : 0);
    cplx<R> s[12];
    SpinorIO<P>::load(hv, g.vh, h, s);
    double2 *dst = out + r * out_rhs_stride + i * 12;
#pragma unroll
    for (int c = 0; c < 12; ++c) dst[c] = make_double2((double)s[c].re, (double)s[c].im);
}

laph_status pack_spinor(const Ctx &c, Operand out, const double *in, int prec, int nrhs, int parity,
                        size_t in_rhs_stride_elems) {
    if (nrhs <= 0) return LAPH_OK;
    const int np = parity < 0 ? 2 : 1;
    const size_t stride = in_rhs_stride_elems ? in_rhs_stride_elems : (size_t)2 * c.g.vh * 12;
    dim3 grid((c.g.vh + kSetupBlock - 1) / kSetupBlock, nrhs, np);
    const double2 *src = reinterpret_cast<const double2 *>(in);
    if (prec == LAPH_F64)
        hipLaunchKernelGGL(pack_kernel<F64>, grid, dim3(kSetupBlock), 0, c.stream, c.g, out, src, stride, parity, np);
    else if (prec == LAPH_F32)
        hipLaunchKernelGGL(pack_kernel<F32>, grid, dim3(kSetupBlock), 0, c.stream, c.g, out, src, stride, parity, np);
    else
        hipLaunchKernelGGL(pack_kernel<F16N>, grid, dim3(kSetupBlock), 0, c.stream, c.g, out, src, stride, parity, np);
    return check_launch("pack_kernel");
}

laph_status unpack_spinor(const Ctx &c, double *out, Operand in, int prec, int nrhs, int parity,
                          size_t out_rhs_stride_elems) {
    if (nrhs <= 0) return LAPH_OK;
    const int np = parity < 0 ? 2 : 1;
    const size_t stride = out_rhs_stride_elems ? out_rhs_stride_elems : (size_t)2 * c.g.vh * 12;
    dim3 grid((c.g.vh + kSetupBlock - 1) / kSetupBlock, nrhs, np);
    double2 *dst = reinterpret_cast<double2 *>(out);
    if (prec == LAPH_F64)
        hipLaunchKernelGGL(unpack_kernel<F64>, grid, dim3(kSetupBlock), 0, c.stream, c.g, dst, stride, in, parity, np);
    else if (prec == LAPH_F32)
        hipLaunchKernelGGL(unpack_kernel<F32>, grid, dim3(kSetupBlock), 0, c.stream, c.g, dst, stride, in, parity, np);
    else
        hipLaunchKernelGGL(unpack_kernel<F16N>, grid, dim3(kSetupBlock), 0, c.stream, c.g, dst, stride, in, parity,
                           np);
    return check_launch("unpack_kernel");
}

}  // namespace laph
