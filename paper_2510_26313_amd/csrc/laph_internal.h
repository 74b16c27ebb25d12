// Internal definitions shared by the HIP kernels and the host code of liblaph.
//
// Internal field layouts (all even-odd, structure-of-arrays over the Vh = V/2
// sites of one parity, checkerboard index h = (x + Lx (y + Ly (z + Lz t))) >> 1):
//
//   spinor half-vector (one parity, one RHS), spin-colour component c = 3 s + a
//     F64 : [12][Vh] double2                 192 B/site
//     F32 : [6][Vh]  float4 (components 2j, 2j+1)   96 B/site
//     F16N: [3][Vh]  8 x binary16 (components 4j..4j+3), then [Vh] FP32 norm   52 B/site
//   every half-vector starts on a 256-byte boundary; a full field is
//   [rhs][parity][half-vector], a parity-only field [rhs][half-vector].
//
//   gauge, per parity p and direction mu (links U_mu(x) of the sites x of parity p)
//     F64 : [9][Vh] double2 (row-major 3x3)
//     F32 : [3][Vh] float4  (rows 0 and 1; row 2 = conj(row0 x row1), det U = 1)
//     F16 : [Vh] 8 x binary16 (row 0, row 1 col 0) + [Vh] 4 x binary16 (row 1 cols 1, 2)
//
//   clover blocks, per parity and chiral block (spins {0,1} or {2,3}): a Hermitian
//   6x6 matrix packed as 36 reals: 6 real diagonal entries, then the 15 complex
//   entries below the diagonal in the order (1,0),(2,0),(2,1),(3,0),...,(5,4)
//     F64 : [18][Vh] double2,  F32 : [9][Vh] float4
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/laph.h"

namespace laph {

// ---------------------------------------------------------------------------
// complex arithmetic
// ---------------------------------------------------------------------------
template <class R>
struct cplx {
    R re, im;
};

template <class R>
__host__ __device__ __forceinline__ cplx<R> mk(R a, R b) { return cplx<R>{a, b}; }
template <class R>
__host__ __device__ __forceinline__ cplx<R> operator+(cplx<R> a, cplx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R>
__host__ __device__ __forceinline__ cplx<R> operator-(cplx<R> a, cplx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R>
__host__ __device__ __forceinline__ cplx<R> operator*(cplx<R> a, cplx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R>
__host__ __device__ __forceinline__ cplx<R> operator*(R s, cplx<R> a) { return {s * a.re, s * a.im}; }
template <class R>
__host__ __device__ __forceinline__ cplx<R> conj(cplx<R> a) { return {a.re, -a.im}; }
// multiply by +i, -i
template <class R>
__host__ __device__ __forceinline__ cplx<R> mul_i(cplx<R> a) { return {-a.im, a.re}; }
template <class R>
__host__ __device__ __forceinline__ cplx<R> mul_mi(cplx<R> a) { return {a.im, -a.re}; }
// fused multiply-add in the operands' precision (host and device)
__host__ __device__ __forceinline__ float ffma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__host__ __device__ __forceinline__ double ffma(double a, double b, double c) { return __builtin_fma(a, b, c); }

// a += b * c ; a += conj(b) * c.  Written as a sum of products rather than a
// chain of four fused multiply-adds: the chained form lets the scheduler keep
// more independent chains in flight and roughly doubles the stencil kernels'
// VGPRs (fewer waves to hide the neighbour gathers), which costs more than the
// extra adds.
template <class R>
__host__ __device__ __forceinline__ void cmac(cplx<R> &a, cplx<R> b, cplx<R> c) {
    a.re += b.re * c.re - b.im * c.im;
    a.im += b.re * c.im + b.im * c.re;
}
template <class R>
__host__ __device__ __forceinline__ void cmac_conj(cplx<R> &a, cplx<R> b, cplx<R> c) {
    a.re += b.re * c.re + b.im * c.im;
    a.im += b.re * c.im - b.im * c.re;
}
// The same as chains of four fused multiply-adds: fewer instructions, but each
// chain is serial, so the scheduler keeps more of them in flight; used where the
// caller bounds the live registers (the LDS stencil form's fences).
template <class R>
__host__ __device__ __forceinline__ void cfma(cplx<R> &a, cplx<R> b, cplx<R> c) {
    a.re = ffma(b.re, c.re, a.re);
    a.re = ffma(-b.im, c.im, a.re);
    a.im = ffma(b.re, c.im, a.im);
    a.im = ffma(b.im, c.re, a.im);
}
template <class R>
__host__ __device__ __forceinline__ void cfma_conj(cplx<R> &a, cplx<R> b, cplx<R> c) {
    a.re = ffma(b.re, c.re, a.re);
    a.re = ffma(b.im, c.im, a.re);
    a.im = ffma(b.re, c.im, a.im);
    a.im = ffma(-b.im, c.re, a.im);
}
// b * c and conj(b) * c (one multiply and three fused multiply-adds)
template <class R>
__host__ __device__ __forceinline__ cplx<R> cmul1(cplx<R> b, cplx<R> c) {
    return {ffma(-b.im, c.im, b.re * c.re), ffma(b.im, c.re, b.re * c.im)};
}
template <class R>
__host__ __device__ __forceinline__ cplx<R> cmul1_conj(cplx<R> b, cplx<R> c) {
    return {ffma(b.im, c.im, b.re * c.re), ffma(-b.im, c.re, b.re * c.im)};
}
// a + s * b for real s
template <class R>
__host__ __device__ __forceinline__ cplx<R> caxpy(R s, cplx<R> b, cplx<R> a) {
    return {ffma(s, b.re, a.re), ffma(s, b.im, a.im)};
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
struct Geom {
    int lx, ly, lz, lt;
    int lxh;        // lx / 2
    int vh;         // sites per parity
    int vs_h;       // sites per parity on one timeslice (lx ly lz / 2)
    int antiperiodic;
};

__device__ __forceinline__ void site_coords(const Geom &g, int parity, int h, int &x, int &y, int &z, int &t) {
    int xh = h % g.lxh;
    int r = h / g.lxh;
    y = r % g.ly;
    r /= g.ly;
    z = r % g.lz;
    t = r / g.lz;
    x = 2 * xh + ((parity + y + z + t) & 1);
}

__device__ __forceinline__ int cb_index(const Geom &g, int x, int y, int z, int t) {
    return (x + g.lx * (y + g.ly * (z + g.lz * t))) >> 1;
}

// A cyclic range [lo, lo + n) mod vh of checkerboard site indices.  In either parity
// the sites of one timeslice t are h = t vs_h .. (t + 1) vs_h - 1, so a slab of
// consecutive timeslices is one such range.  n <= 0: every site.
struct SiteWindow {
    int lo = 0;
    int n = 0;
};

__host__ __device__ inline bool in_window(const SiteWindow &w, int h, int vh) {
    if (w.n <= 0) return true;
    int d = h - w.lo;
    if (d < 0) d += vh;
    return d < w.n;
}

// no site of [h0, h0 + cnt) (all inside 0 .. vh-1) lies in the window
__host__ __device__ inline bool block_outside(const SiteWindow &w, int h0, int cnt, int vh) {
    if (w.n <= 0) return false;
    int d = h0 - w.lo;
    if (d < 0) d += vh;
    return d >= w.n && d + cnt <= vh;
}

// the timeslices t0 - k .. t0 + k (periodic in t); every site when they cover the lattice
inline SiteWindow slab_window(const Geom &g, int t0, int k) {
    SiteWindow w;
    if (2 * k + 1 >= g.lt) return w;
    w.lo = ((t0 - k) % g.lt + g.lt) % g.lt * g.vs_h;
    w.n = (2 * k + 1) * g.vs_h;
    return w;
}

// ---------------------------------------------------------------------------
// precisions
// ---------------------------------------------------------------------------
struct F64 {
    using real = double;
    static constexpr int id = LAPH_F64;
};
struct F32 {
    using real = float;
    static constexpr int id = LAPH_F32;
};
struct F16N {
    using real = float;
    static constexpr int id = LAPH_F16N;
};

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));

inline size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

inline size_t hv_bytes(int prec, size_t vh) {
    size_t per = prec == LAPH_F64 ? 192 : (prec == LAPH_F32 ? 96 : 52);
    return round256(per * vh);
}

// ---------------------------------------------------------------------------
// spinor site load / store (one site of one half-vector)
// ---------------------------------------------------------------------------
template <class P>
struct SpinorIO;

// load_unscaled: the stored values before the per-site norm (FP16N codes as FP32)
// and that norm (1 for FP64 / FP32), so a linear consumer can apply the norm once
// to a smaller result.
template <>
struct SpinorIO<F64> {
    static constexpr bool kNorm = false;
    static __device__ __forceinline__ void load_unscaled(const char *hv, int vh, int h, cplx<double> (&s)[12],
                                                         double &n) {
        load(hv, vh, h, s);
        n = 1.0;
    }
    static __device__ __forceinline__ void load(const char *hv, int vh, int h, cplx<double> (&s)[12]) {
        const double2 *p = reinterpret_cast<const double2 *>(hv);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            double2 v = p[(size_t)c * vh + h];
            s[c] = {v.x, v.y};
        }
    }
    // one chiral block: components 6 blk .. 6 blk + 5 (spins 2 blk and 2 blk + 1)
    static __device__ __forceinline__ void load_block(const char *hv, int vh, int h, int blk, cplx<double> (&s)[6]) {
        const double2 *p = reinterpret_cast<const double2 *>(hv) + (size_t)6 * blk * vh;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            double2 v = p[(size_t)c * vh + h];
            s[c] = {v.x, v.y};
        }
    }
    static __device__ __forceinline__ void store(char *hv, int vh, int h, const cplx<double> (&s)[12]) {
        double2 *p = reinterpret_cast<double2 *>(hv);
#pragma unroll
        for (int c = 0; c < 12; ++c) p[(size_t)c * vh + h] = make_double2(s[c].re, s[c].im);
    }
};

template <>
struct SpinorIO<F32> {
    static constexpr bool kNorm = false;
    static __device__ __forceinline__ void load_unscaled(const char *hv, int vh, int h, cplx<float> (&s)[12],
                                                         float &n) {
        load(hv, vh, h, s);
        n = 1.f;
    }
    static __device__ __forceinline__ void load(const char *hv, int vh, int h, cplx<float> (&s)[12]) {
        const float4 *p = reinterpret_cast<const float4 *>(hv);
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            float4 v = p[(size_t)j * vh + h];
            s[2 * j] = {v.x, v.y};
            s[2 * j + 1] = {v.z, v.w};
        }
    }
    static __device__ __forceinline__ void store(char *hv, int vh, int h, const cplx<float> (&s)[12]) {
        float4 *p = reinterpret_cast<float4 *>(hv);
#pragma unroll
        for (int j = 0; j < 6; ++j)
            p[(size_t)j * vh + h] = make_float4(s[2 * j].re, s[2 * j].im, s[2 * j + 1].re, s[2 * j + 1].im);
    }
};

template <>
struct SpinorIO<F16N> {
    static constexpr bool kNorm = true;
    static __device__ __forceinline__ void load_codes(const char *hv, int vh, int h, half8 (&q)[3], float &n) {
        const half8 *p = reinterpret_cast<const half8 *>(hv);
        n = reinterpret_cast<const float *>(hv + (size_t)48 * vh)[h];
#pragma unroll
        for (int j = 0; j < 3; ++j) q[j] = p[(size_t)j * vh + h];
    }
    static __device__ __forceinline__ void load_unscaled(const char *hv, int vh, int h, cplx<float> (&s)[12],
                                                         float &n) {
        const half8 *p = reinterpret_cast<const half8 *>(hv);
        n = reinterpret_cast<const float *>(hv + (size_t)48 * vh)[h];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            half8 v = p[(size_t)j * vh + h];
#pragma unroll
            for (int k = 0; k < 4; ++k) s[4 * j + k] = {(float)v[2 * k], (float)v[2 * k + 1]};
        }
    }
    static __device__ __forceinline__ void load(const char *hv, int vh, int h, cplx<float> (&s)[12]) {
        const half8 *p = reinterpret_cast<const half8 *>(hv);
        const float n = reinterpret_cast<const float *>(hv + (size_t)48 * vh)[h];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            half8 v = p[(size_t)j * vh + h];
#pragma unroll
            for (int k = 0; k < 4; ++k) s[4 * j + k] = {(float)v[2 * k] * n, (float)v[2 * k + 1] * n};
        }
    }
    static __device__ __forceinline__ void store(char *hv, int vh, int h, const cplx<float> (&s)[12]) {
        float n = 0.f;
#pragma unroll
        for (int c = 0; c < 12; ++c) n = fmaxf(n, fmaxf(fabsf(s[c].re), fabsf(s[c].im)));
        const float inv = n > 0.f ? 1.0f / n : 0.f;
        half8 *p = reinterpret_cast<half8 *>(hv);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            half8 v;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                v[2 * k] = (_Float16)(s[4 * j + k].re * inv);
                v[2 * k + 1] = (_Float16)(s[4 * j + k].im * inv);
            }
            p[(size_t)j * vh + h] = v;
        }
        reinterpret_cast<float *>(hv + (size_t)48 * vh)[h] = n;
    }
};

// ---------------------------------------------------------------------------
// gauge link load (one link)
// ---------------------------------------------------------------------------
struct GaugePtrs {
    // [parity][mu] base pointers of the per-(parity, mu) arrays
    const char *f64[2][4];
    const char *f32[2][4];
    const char *f16a[2][4];
    const char *f16b[2][4];
};

template <class R>
__device__ __forceinline__ void reconstruct_row2(cplx<R> (&u)[9]) {
    // row2 = conj(row0 x row1)
    u[6] = conj(u[1] * u[5] - u[2] * u[4]);
    u[7] = conj(u[2] * u[3] - u[0] * u[5]);
    u[8] = conj(u[0] * u[4] - u[1] * u[3]);
}

template <class P>
struct GaugeIO;

template <>
struct GaugeIO<F64> {
    static __device__ __forceinline__ void load(const GaugePtrs &g, int parity, int mu, int vh, int h,
                                                cplx<double> (&u)[9]) {
        const double2 *p = reinterpret_cast<const double2 *>(g.f64[parity][mu]);
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            double2 v = p[(size_t)k * vh + h];
            u[k] = {v.x, v.y};
        }
    }
};

template <>
struct GaugeIO<F32> {
    static __device__ __forceinline__ void load(const GaugePtrs &g, int parity, int mu, int vh, int h,
                                                cplx<float> (&u)[9]) {
        const float4 *p = reinterpret_cast<const float4 *>(g.f32[parity][mu]);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            float4 v = p[(size_t)j * vh + h];
            u[2 * j] = {v.x, v.y};
            u[2 * j + 1] = {v.z, v.w};
        }
        reconstruct_row2(u);
    }
};

template <>
struct GaugeIO<F16N> {
    static __device__ __forceinline__ void load(const GaugePtrs &g, int parity, int mu, int vh, int h,
                                                cplx<float> (&u)[9]) {
        half8 a = reinterpret_cast<const half8 *>(g.f16a[parity][mu])[h];
        half4 b = reinterpret_cast<const half4 *>(g.f16b[parity][mu])[h];
#pragma unroll
        for (int k = 0; k < 4; ++k) u[k] = {(float)a[2 * k], (float)a[2 * k + 1]};
        u[4] = {(float)b[0], (float)b[1]};
        u[5] = {(float)b[2], (float)b[3]};
        reconstruct_row2(u);
    }
};

// ---------------------------------------------------------------------------
// packed Hermitian 6x6 clover blocks
// ---------------------------------------------------------------------------
template <class P>
struct CloverIO;

template <>
struct CloverIO<F64> {
    // base: [block 2][18][vh] double2 for one parity
    static __device__ __forceinline__ void load(const char *base, int block, int vh, int h, double (&m)[36]) {
        const double2 *p = reinterpret_cast<const double2 *>(base) + (size_t)block * 18 * vh;
#pragma unroll
        for (int k = 0; k < 18; ++k) {
            double2 v = p[(size_t)k * vh + h];
            m[2 * k] = v.x;
            m[2 * k + 1] = v.y;
        }
    }
};

template <class P>
struct CloverIO {
    // F32 and F16N paths: [block 2][9][vh] float4 for one parity
    static __device__ __forceinline__ void load(const char *base, int block, int vh, int h, float (&m)[36]) {
        const float4 *p = reinterpret_cast<const float4 *>(base) + (size_t)block * 9 * vh;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            float4 v = p[(size_t)k * vh + h];
            m[4 * k] = v.x;
            m[4 * k + 1] = v.y;
            m[4 * k + 2] = v.z;
            m[4 * k + 3] = v.w;
        }
    }
};

// y = M x for a packed Hermitian 6x6 M (optionally with diag_shift added to the diagonal)
template <class R>
__device__ __forceinline__ void herm6_apply(const R (&m)[36], const cplx<R> *x, cplx<R> *y, R diag_shift = R(0)) {
#pragma unroll
    for (int i = 0; i < 6; ++i) y[i] = (m[i] + diag_shift) * x[i];
    int k = 0;
#pragma unroll
    for (int i = 1; i < 6; ++i) {
#pragma unroll
        for (int j = 0; j < i; ++j) {
            cplx<R> l = {m[6 + 2 * k], m[7 + 2 * k]};
            cmac(y[i], l, x[j]);
            cmac_conj(y[j], l, x[i]);
            ++k;
        }
    }
}

// herm6_apply with the multiply-adds as fused chains (see cfma)
template <class R>
__device__ __forceinline__ void herm6_apply_fma(const R (&m)[36], const cplx<R> *x, cplx<R> *y) {
#pragma unroll
    for (int i = 0; i < 6; ++i) y[i] = m[i] * x[i];
    int k = 0;
#pragma unroll
    for (int i = 1; i < 6; ++i) {
#pragma unroll
        for (int j = 0; j < i; ++j) {
            cplx<R> l = {m[6 + 2 * k], m[7 + 2 * k]};
            cfma(y[i], l, x[j]);
            cfma_conj(y[j], l, x[i]);
            ++k;
        }
    }
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
// Workgroups are dispatched round-robin over the 8 XCDs of the chip.  Remap so
// that the workgroups one XCD receives form a contiguous range of logical ids:
// the RHS tiles of one site block then run on the same XCD (shared L2).
__device__ __forceinline__ int xcd_logical_block() {
    const int n = gridDim.x;   // launches pad the grid to a multiple of 8
    const int per = n >> 3;
    const int id = blockIdx.x;
    return (id & 7) * per + (id >> 3);
}

inline int pad8(int n) { return (n + 7) & ~7; }

}  // namespace laph
