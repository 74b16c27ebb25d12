// FP64 reductions and the streaming copy of the boundary calls.
//
//  * stage partials -> per-RHS inner products (laph_apply_stage): the fused
//    stencil stages leave one FP64 partial sum per site block, RHS and quantity;
//    one block per (RHS, quantity) adds them in a fixed order.
//  * the mass gradient of the differentiable solve (laph_mass_gradient): with
//    X = D(m0)^-1 B and dD/dm0 = 1, a loss L(X) has dL/dm0 = -sum_r Re<Z_r, X_r>
//    for the adjoint solutions Z = D^-dagger (dL/dX), the convention
//    grad = dL/dRe + i dL/dIm of the complex cotangent.  Re<Z, X> of two
//    complex128 arrays is the real dot product of their (re, im) pairs.
//  * a plain streaming copy (laph_stream_copy): the rate a bandwidth-bound
//    kernel of this library can reach, the reference its roofline fractions
//    are also quoted against.
//
// Every sum runs in a fixed order (a fixed grid-stride pattern per thread,
// wave shuffles, a block's waves through LDS, then one block over the block
// partials), so results are reproducible run to run.
#include "laph_reduce.h"

namespace laph {

constexpr int kRB = 256;

// Sum of one value per thread over a block of kRB threads, fixed order; the
// result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[kRB / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kRB / 64; ++w) s += red[w];
    return s;
}

// out[r * 3 + q] = sum_{sb < nsb} partials[(r * 3 + q) * pstride + sb]; one block per (r, q)
__global__ __launch_bounds__(kRB) void sum_partials_kernel(const double *partials, int pstride, int nsb, int nq,
                                                           double *out) {
    const int r = blockIdx.x / nq, q = blockIdx.x % nq;
    const double *p = partials + ((size_t)r * 3 + q) * pstride;
    double s = 0;
    for (int i = threadIdx.x; i < nsb; i += kRB) s += p[i];
    s = block_sum(s);
    if (threadIdx.x == 0) out[(size_t)r * 3 + q] = s;
}

laph_status sum_stage_partials(const Ctx &c, const double *partials, int pstride, int nsb, int nrhs, int nq,
                               double *out) {
    if (nrhs <= 0 || nq <= 0) return LAPH_OK;
    hipLaunchKernelGGL(sum_partials_kernel, dim3(nrhs * nq), dim3(kRB), 0, c.stream, partials, pstride, nsb, nq, out);
    return check_launch("sum_partials_kernel");
}

// partial[b] = sum over the elements i = b*kRB + t + k*stride of Re(conj(z_i) x_i)
__global__ __launch_bounds__(kRB) void re_dot_partials_kernel(const double2 *z, const double2 *x, size_t n,
                                                              double *partial) {
    const size_t stride = (size_t)gridDim.x * kRB;
    double s0 = 0, s1 = 0;
    size_t i = (size_t)blockIdx.x * kRB + threadIdx.x;
    for (; i + stride < n; i += 2 * stride) {
        const double2 a = z[i], b = x[i], c = z[i + stride], d = x[i + stride];
        s0 = fma(a.x, b.x, s0);
        s0 = fma(a.y, b.y, s0);
        s1 = fma(c.x, d.x, s1);
        s1 = fma(c.y, d.y, s1);
    }
    if (i < n) {
        const double2 a = z[i], b = x[i];
        s0 = fma(a.x, b.x, s0);
        s0 = fma(a.y, b.y, s0);
    }
    const double s = block_sum(s0 + s1);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// out[0] = scale * sum_{b < nb} partial[b]   (one block)
__global__ __launch_bounds__(kRB) void sum_scaled_kernel(const double *partial, int nb, double scale, double *out) {
    double s = 0;
    for (int i = threadIdx.x; i < nb; i += kRB) s += partial[i];
    s = block_sum(s);
    if (threadIdx.x == 0) out[0] = scale * s;
}

laph_status mass_gradient(const Ctx &c, double *g_host, const double *Z, const double *X, size_t n_complex,
                          double *scratch) {
    hipLaunchKernelGGL(re_dot_partials_kernel, dim3(kGradBlocks), dim3(kRB), 0, c.stream,
                       reinterpret_cast<const double2 *>(Z), reinterpret_cast<const double2 *>(X), n_complex, scratch);
    LAPH_TRY(check_launch("re_dot_partials_kernel"));
    hipLaunchKernelGGL(sum_scaled_kernel, dim3(1), dim3(kRB), 0, c.stream, scratch, kGradBlocks, -1.0,
                       scratch + kGradBlocks);
    LAPH_TRY(check_launch("sum_scaled_kernel"));
    LAPH_HIP(hipMemcpyAsync(g_host, scratch + kGradBlocks, sizeof(double), hipMemcpyDeviceToHost, c.stream));
    LAPH_HIP(hipStreamSynchronize(c.stream));
    return LAPH_OK;
}

// dst = src, one 16-byte word per thread, one workgroup per 4 KiB: the grid walks
// the buffer once in dispatch order.  Measured on MI355X (4 GiB): 6.16 TB/s read +
// write, against 4.7-5.5 TB/s for grid-stride loops of 2048-65536 workgroups with
// 1, 4 or 8 words in flight per thread (non-temporal loads or stores changed little).
__global__ __launch_bounds__(kRB) void stream_copy_kernel(uint4 *dst, const uint4 *src, size_t n) {
    const size_t i = (size_t)blockIdx.x * kRB + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

laph_status stream_copy(const Ctx &c, void *dst, const void *src, size_t bytes, int reps, double *ms_host) {
    const size_t n = bytes / 16;
    const size_t want = (n + kRB - 1) / kRB;
    if (want > (size_t)0x7fffffff) return set_error(LAPH_ERR_INVALID, "copy too large for one grid");
    const unsigned grid = (unsigned)(want > 0 ? want : 1);
    auto launch = [&]() {
        hipLaunchKernelGGL(stream_copy_kernel, dim3(grid), dim3(kRB), 0, c.stream, reinterpret_cast<uint4 *>(dst),
                           reinterpret_cast<const uint4 *>(src), n);
        return check_launch("stream_copy_kernel");
    };
    LAPH_TRY(launch());   // warm
    LAPH_HIP(hipEventRecord(c.ev[0], c.stream));
    for (int i = 0; i < reps; ++i) LAPH_TRY(launch());
    LAPH_HIP(hipEventRecord(c.ev[1], c.stream));
    LAPH_HIP(hipEventSynchronize(c.ev[1]));
    float ms = 0;
    LAPH_HIP(hipEventElapsedTime(&ms, c.ev[0], c.ev[1]));
    *ms_host = ms / reps;
    return LAPH_OK;
}

}  // namespace laph
